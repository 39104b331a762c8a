"""Throughput benchmark of the Monte Carlo SPECT transport path on one MI355X.

A step is one pass of the forward hot path over the 128^3 thorax workload
(60 views over 180 degrees, 64x64 pixels at 6 mm, 126-154 keV window, 1e8
photon histories): input staging, transport, tallies.  Inputs are resident in
HBM before timing starts.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--histories N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
N_CU, CLOCK_HZ = 256, 2.4e9
PEAK_LANE_OPS = N_CU * 64 * CLOCK_HZ  # one 32-bit VALU instruction per lane per clock

# Algorithmic work per history: the method's operation table (Philox blocks,
# transcendentals, other 32-bit operations per emission, per tentative
# collision, per Kahn attempt and per real collision), with a Philox4x32-10
# block counted as the 40 instructions it is in the library's gfx950
# assembly (10 rounds x (2 v_mad_u64_u32 + 2 three-way xors, v_bitop3_b32);
# the key schedule is scalar).  Counts come from the kernel's own work
# counters.
OPS_PHILOX = 40
TABLE = {            # (Philox blocks, transcendentals, other operations)
    "emission": (2, 3, 20),          # voxel, position, sqrt/sin/cos direction
    "tentative": (1, 1, 10),         # log flight, move, voxel, accept test
    "kahn_attempt": (1, 0, 0),       # the attempt's Philox block (its test is counted per real collision)
    "real": (0, 3, 40),              # branch, Kahn test, sqrt/sin/cos rotation, energy terms
}


# Forced copies (Sec. 5.2): per copy whose ray is walked to the detector, a
# Philox block (the cone direction), 6 transcendentals (sin, cos and sqrt of
# the rotation, two reciprocals of the Klein-Nishina density, the
# attenuation exponential) and ~60 other operations (rotation, density,
# detector hit and bin, tally); per voxel the walk visits, ~8 (next plane:
# min of three, axis select, parameter and index update, exit test; the
# path-length product) and one 4-byte mu gather from L2.
OPS_PER_RAY = (1, 6, 60)
OPS_PER_VOXEL = 8
BYTES_PER_VOXEL = 4


def table_ops(n_hist, n_tent, n_kahn, n_real, cost=None):
    """Operations of the table for these counts; cost: optional issue cost of
    a Philox block, a transcendental and another operation (full-rate
    slots), else one operation each (a Philox block = OPS_PHILOX)."""
    ph, tr, ot = cost if cost else (OPS_PHILOX, 1.0, 1.0)
    n = {"emission": n_hist, "tentative": n_tent, "kahn_attempt": n_kahn, "real": n_real}
    return sum(n[k] * (p * ph + t * tr + o * ot) for k, (p, t, o) in TABLE.items())


# HBM traffic of one transport launch on the headline workload, from rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by what the same
# counters read for a plain 1 GiB device copy (FETCH x2.0, WRITE x1.0); keyed
# by a hash of the kernel sources so a changed kernel reports null.
COPY_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC_KIB = {"a6209a920f84733f": {"fetch": 5967.5, "write": 4983.19}}
# rocprofv3 --pmc SQ_INSTS_VALU of the same launch (and the dispatch time of
# that run), keyed like the traffic
VALU_COUNTERS = {"a6209a920f84733f": {"workload": "thorax_128", "SQ_INSTS_VALU": 1.90174e9,
                                      "kernel_ms": 3.8077}}


def kernel_source_hash() -> str:
    import hashlib
    m = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2105_13324_amd", "csrc")
    for f in ("history.h", "transport.hip", "mc_internal.h"):
        with open(os.path.join(d, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def traffic_bytes():
    t = TRAFFIC_KIB.get(kernel_source_hash())
    if t is None:
        return None
    return 1024.0 * (t["fetch"] * COPY_SCALE["fetch"] + t["write"] * COPY_SCALE["write"])


PROBE_CLASSES = ["mad_u64", "xor_add", "fma", "log", "sin", "sqrt", "rcp", "philox_block"]


def issue_rates(torch, blocks=None, iters=20000):
    """Sustained issue rate of each instruction class the transport uses, from
    the probe kernels (libmcprobe.so): eight independent chains per lane, no
    memory traffic, eight waves per SIMD.  Returns the cost of one
    lane-operation of each class in full-rate lane slots (xor/add = 1) and the
    measured full-rate rate in lane-ops/s.  Loop bodies (from the probes'
    gfx950 assembly): mad64 8 v_mad_u64_u32 + 8 v_xor; xor 8 v_xor + 8 v_add;
    fma 8 v_fmaak; each transcendental 8 of it + 8 v_mul; the Philox probe
    one ten-round block (20 v_mad_u64_u32, 20 v_bitop3) per eighth iteration."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2105_13324_amd", "libmcprobe.so"))
    lib.mc_probe_issue.argtypes = [C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_float), C.c_void_p]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = blocks or n_cu * 8
    scratch = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    ms = (C.c_float * 8)()
    rc = lib.mc_probe_issue(blocks, iters, scratch.data_ptr(), ms,
                            torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise RuntimeError(f"mc_probe_issue failed ({rc})")
    t = dict(zip(PROBE_CLASSES, [float(x) for x in ms]))
    lanes = blocks * 256 * iters
    full = 16 * lanes / (t["xor_add"] / 1e3)           # full-rate lane-ops/s
    slot = t["xor_add"] / 16                            # ms per (lane-op x lanes x iters)
    cost = {"xor_add": 1.0, "fma": t["fma"] / (8 * slot),
            "mad_u64": (t["mad_u64"] - 8 * slot) / (8 * slot)}
    mul = cost["fma"]                                   # v_mul_f32 issues like v_fma
    for k in ("log", "sin", "sqrt", "rcp"):
        cost[k] = (t[k] - 8 * mul * slot) / (8 * slot)
    # one Philox block per eighth iteration: its cost in full-rate slots
    cost["philox_block"] = t["philox_block"] / (slot * (iters // 8) / iters)
    return {"full_rate_lane_ops_per_s": full, "peak_nominal_lane_ops_per_s": PEAK_LANE_OPS,
            "cost_in_full_rate_slots": cost, "probe_ms": t, "blocks": blocks, "iters": iters}


def transport_roofline(sim, k_ms, rates=None, kernel="k_transport", counters_key=None):
    """ALU roofline of one transport launch from the work counters of all its
    problems.  frac: the table's operations (one per instruction, a Philox
    block = 40) per second over the nominal peak, 256 CU x 64 lanes x
    2.4 GHz.  With measured issue rates (issue_rates): the shortest time the
    same operations take at the rates the probes sustain (full-rate slots,
    a v_mad_u64_u32 and a transcendental as measured) against the kernel
    time, and, from the committed counter profile of this kernel build, the
    VALU instructions it actually issued."""
    cnt = sim.counters.cpu().numpy().astype(np.float64).sum(axis=0)
    n_tent, n_real, n_kahn, n_hist = cnt[:4]
    ops = table_ops(n_hist, n_tent, n_kahn, n_real)
    achieved = ops / (k_ms / 1e3)
    out = {"bound": "alu", "kernel": kernel, "kernel_ms": k_ms,
           "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
           "unit": "Tops/s (32-bit lane ops, one per instruction)", "frac": achieved / PEAK_LANE_OPS,
           "ops_per_history": ops / n_hist,
           # the same table with a Philox block at 100 (the middle of the
           # 80-120 range of a generic count) instead of its 40 gfx950 instructions
           "frac_philox_100": table_ops(n_hist, n_tent, n_kahn, n_real, cost=(100, 1.0, 1.0))
                              / (k_ms / 1e3) / PEAK_LANE_OPS,
           "op_table": "per history: emission 2 Philox + 3 transcendental + 20; per tentative "
                       "collision 1 Philox + log + 10; per Kahn attempt 1 Philox; per real collision "
                       "3 transcendental + 40; Philox = 40 gfx950 instructions"}
    if rates:
        c = rates["cost_in_full_rate_slots"]
        slots = table_ops(n_hist, n_tent, n_kahn, n_real,
                          cost=(c["philox_block"], np.mean([c[k] for k in ("log", "sin", "sqrt", "rcp")]), 1.0))
        t_min = slots / rates["full_rate_lane_ops_per_s"]
        out["frac_of_measured_op_mix_peak"] = t_min / (k_ms / 1e3)
        out["op_mix_slots_per_history"] = slots / n_hist
    if counters_key:
        pc = VALU_COUNTERS.get(kernel_source_hash())
        if pc is not None and pc.get("workload") == counters_key:
            issued = pc["SQ_INSTS_VALU"] * 64
            out["issue_frac"] = issued / (pc["kernel_ms"] / 1e3) / PEAK_LANE_OPS
            out["issued_valu_per_history"] = pc["SQ_INSTS_VALU"] * 64 / n_hist
    return out


def forced_roofline(sim, k_ms, kernel):
    """ALU roofline of a forced-detection or weighted transport launch: the
    analog table for its histories plus, for forced copies, OPS_PER_RAY per
    walked ray and OPS_PER_VOXEL per visited voxel (counters 4 and 5), over
    the nominal peak."""
    cnt = sim.counters.cpu().numpy().astype(np.float64).sum(axis=0)
    n_tent, n_real, n_kahn, n_hist, rays, voxels = cnt[:6]
    ops = table_ops(n_hist, n_tent, n_kahn, n_real)
    ph, tr, ot = OPS_PER_RAY
    ops += rays * (ph * OPS_PHILOX + tr + ot) + voxels * OPS_PER_VOXEL
    achieved = ops / (k_ms / 1e3)
    out = {"bound": "alu", "kernel": kernel, "kernel_ms": k_ms, "achieved": achieved / 1e12,
           "peak": PEAK_LANE_OPS / 1e12, "unit": "Tops/s (32-bit lane ops, one per instruction)",
           "frac": achieved / PEAK_LANE_OPS, "ops_per_history": ops / n_hist}
    if rays:
        out.update({"rays_per_history": rays / n_hist, "voxels_per_ray": voxels / rays,
                    "ray_unit": "voxel crossing: %d ops, %d B (mu gather, L2)" % (OPS_PER_VOXEL, BYTES_PER_VOXEL),
                    "crossings_per_s": voxels / (k_ms / 1e3),
                    "mu_gather_GBps": voxels * BYTES_PER_VOXEL / (k_ms / 1e3) / 1e9})
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, mc, dp, torch, full_limit_s: float = 60.0, target_s: float = 12.0):
    """The FP64 oracle on the host cores.  When the whole workload fits in
    full_limit_s of wall time (estimated from a 1e6-history run) it is timed
    on the whole workload, and that run is also the reference of the parity
    block; otherwise on a bounded sample, and the parity block is left out."""
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    n0 = min(10 ** 6, prob.n_histories)
    t = time.perf_counter()
    oracle.simulate(prob.with_(n_histories=n0), n_threads=cores)
    dt0 = time.perf_counter() - t
    parity = None
    if dt0 * prob.n_histories / n0 <= full_limit_s:
        n = prob.n_histories
        t = time.perf_counter()
        o = oracle.simulate(prob, n_threads=cores, want_triplets=True,
                            trip_cap=max(1 << 20, n // 1000))
        dt = time.perf_counter() - t
        sample = f"the whole workload ({n} histories, {prob.n_views} views)"
        parity = headline_parity(prob, o, mc, dp, torch, cores)
    else:
        n = int(min(max(n0, n0 * target_s / max(dt0, 1e-3)), prob.n_histories))
        t = time.perf_counter()
        oracle.simulate(prob.with_(n_histories=n), n_threads=cores)
        dt = time.perf_counter() - t
        sample = f"first {n} histories of the same workload ({prob.n_views} views)"
    return ({"value": n / dt, "unit": "histories/s", "cores": cores, "kind": "oracle",
             "cpu_model": host_cpu_model(),
             "sample": f"{sample}, {dt:.1f} s wall on {cores} threads; the oracle's plain "
                       f"Woodcock walk (every history followed to the grid edge), FP64"},
            parity)


def headline_parity(prob, o, mc, dp, torch, cores, n_replay=100_000):
    """Per-result errors of the GPU run against the oracle's run of the same
    workload: relative error of the window total, of each class, of each
    fate count and energy; tallied histories on one side only (the transport
    kernel's event list against the oracle's tallied list); identical (fate,
    bin, scatter count) fraction over n_replay ids drawn with numpy PCG64(7)."""
    import oracle
    T = int(o["fates"][5])
    sim = mc.Simulator(dp, want_sq=False, event_capacity=2 * T + 1024)
    sim.run()
    torch.cuda.synchronize()
    ev = sim.events_numpy()
    tally = mc.tally_float(sim.tally).reshape(prob.tally_shape)
    fates = sim.fates.cpu().numpy()[0]
    energy = sim.energy.cpu().numpy()[0].astype(np.float64) / mc.Q23
    gk = ev["work"].astype(np.int64) * (1 << 32) + ev["bin"].astype(np.int64)
    ok = o["trip_g"].astype(np.int64) * (1 << 32) + o["trip_j"].astype(np.int64)
    flipped = int(len(np.setdiff1d(gk, ok)) + len(np.setdiff1d(ok, gk)))
    rel = lambda a, b: float(abs(a - b) / max(abs(b), 1.0))
    rng = np.random.Generator(np.random.PCG64(7))
    N, V = prob.n_histories, prob.n_views
    g = np.sort(rng.choice(N, size=min(n_replay, N), replace=False))
    q, r = divmod(N, V)
    view = np.where(g < r * (q + 1), g // (q + 1), r + (g - r * (q + 1)) // q).astype(np.int32)
    hist = np.where(g < r * (q + 1), g % (q + 1), (g - r * (q + 1)) % q).astype(np.uint64)
    a = mc.replay(dp, view, hist)
    b = oracle.replay(prob, view, hist, n_threads=cores)
    same = ((a["fate"] == b["fate"]) & (a["iu"] == b["iu"]) & (a["iv"] == b["iv"])
            & (a["n_scatter"] == b["n_scatter"]))
    return {"reference": "FP64 oracle, same workload and random streams",
            "tallied_histories": T, "tallied_on_one_side_only": flipped,
            "window_total_rel": rel(tally.sum(), o["tally"].sum()),
            "primary_rel": rel(tally[:, 0].sum(), o["tally"][:, 0].sum()),
            "scatter_rel": rel(tally[:, 1].sum(), o["tally"][:, 1].sum()),
            "bin_l1_rel": float(np.abs(tally - o["tally"]).sum() / max(o["tally"].sum(), 1.0)),
            "fates_max_rel": max(rel(fates[i], o["fates"][i]) for i in range(7)),
            "energy_max_rel": max(rel(energy[i], o["energy"][i]) for i in range(3)),
            "replay_identical": float(same.mean()), "replayed": int(len(same)),
            "replay_ids": "numpy PCG64(7), without replacement"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=float, default=1e8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="time only the headline workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 / 1e9-history form")
    ap.add_argument("--only-form", choices=["forced_detection", "batched", "large_mlem", "adjoint"],
                    default=None,
                    help="time only this side form (forced_detection: forced detection and "
                         "its convolution-based form; batched: the 32-thorax graph; large_mlem: "
                         "the 256^3 thorax with response matrices and MLEM; adjoint: the "
                         "adjoint step on the 128^3 cube) and print its record; for profiling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only run the instruction issue-rate probes and print their record")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the transport path is built and timed on a single "
              "MI355X (multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        # a plain copy of known size: 2^30 bytes read, 2^30 bytes written
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    if args.issue_probe:
        rec = issue_rates(torch)
        # the same probes at 1-4 waves per SIMD: how much of each class's rate
        # survives without the latency hiding of eight resident waves
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        rec["by_waves_per_simd"] = {w: issue_rates(torch, blocks=n_cu * w)["probe_ms"]
                                    for w in (1, 2, 3, 4)}
        print(json.dumps(rec))
        return
    import phantoms
    import paper_2105_13324_amd as mc
    if args.only_form:
        fn = {"forced_detection": fd_form, "batched": batched_form, "large_mlem": large_form,
              "adjoint": adjoint_form}[args.only_form]
        print(json.dumps({"form": args.only_form, **fn(mc, torch, args.steps)}))
        return

    n_hist = int(args.histories)
    prob = phantoms.thorax_128(n_hist)
    dp = mc.to_device(prob)
    timers = [mc.KernelTimer() for _ in range(max(args.steps, 1))]
    sim = mc.Simulator(dp, want_sq=True)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        sim.run()
    torch.cuda.synchronize()
    sim.check_status()

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(args.steps):
        # the library records timers[k] around its transport kernel on this stream
        sim.run(kernel_events=timers[k].handles)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    kernel_ms = [t.elapsed_ms() for t in timers[:args.steps]]
    st = sim.check_status()

    ms_per_step = total_ms / args.steps
    value = n_hist / (ms_per_step / 1e3)
    cnt = sim.counters.cpu().numpy()[0].astype(np.float64)
    fates = sim.fates.cpu().numpy()[0]
    k_ms = float(np.mean(kernel_ms))
    rates = issue_rates(torch)
    roofline = transport_roofline(sim, k_ms, rates, counters_key="thorax_128")
    roofline["traffic"] = traffic_bytes()
    roofline["traffic_unit"] = "bytes per launch (HBM + MALL, from FETCH_SIZE/WRITE_SIZE)"
    rec = {
        "metric": "photon histories/s (128^3 thorax, 60 views) + adjoint μ-grad histories/s",
        "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "thorax_128: 128^3 x 3 mm seeded ellipsoid thorax, 60 views over "
                               "180 deg, 64x64 x 6 mm, 126-154 keV, alpha 2 deg",
                   "histories": n_hist, "views": prob.n_views, "grid": [prob.nx, prob.ny, prob.nz]},
        "roofline": roofline,
        "per_history": {"tentative": cnt[0] / cnt[3], "real": cnt[1] / cnt[3],
                        "kahn_attempts": cnt[2] / cnt[3],
                        "tallied_fraction": float(fates[5]) / cnt[3]},
        "status": int(st[0]),
        "wall_s": wall,
        "issue_rates": {"full_rate_lane_ops_per_s": rates["full_rate_lane_ops_per_s"],
                        "cost_in_full_rate_slots": rates["cost_in_full_rate_slots"]},
    }
    if not args.no_extra:
        rec["forms"] = extra_forms(mc, torch, args, rates)
        a = rec["forms"].get("adjoint")
        if a:
            rec["adjoint_histories_per_s"] = a["value"]
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["parity"] = cpu_baseline(prob, mc, dp, torch)
    print(json.dumps(rec))


def timed(torch, fn, steps):
    """Mean ms of fn() over steps runs, bracketed by device syncs and events."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def extra_forms(mc, torch, args, rates=None):
    """Throughput of the other forms: the point-source cube, the batched graph
    launch over 32 uneven thoraxes, the adjoint (forward with event list +
    replaying gradient) on the 128^3 x 1 mm cube, forced detection on the
    128^3 thorax, and the large workload with reconstruction."""
    import phantoms
    out = {}
    steps = max(args.steps, 1)
    # plain, point source in a 64^3 water cube, 1e6 histories
    p1 = phantoms.point_cube_64(10 ** 6)
    s1 = mc.Simulator(mc.to_device(p1), want_sq=True)
    s1.run()
    ms_eager = timed(torch, s1.run, steps)
    g1 = mc.GraphRunner(s1)
    g1.replay()
    ms = timed(torch, g1.replay, steps)
    out["point_cube_64"] = {"value": p1.n_histories / (ms / 1e3), "unit": "histories/s",
                            "ms_per_step": ms, "eager_ms_per_step": ms_eager,
                            "histories": p1.n_histories, "launch": "hipGraph replay of one call"}
    forms = [("batched", lambda: batched_form(mc, torch, steps, rates)),
             ("adjoint", lambda: adjoint_form(mc, torch, steps, rates)),
             ("forced_detection", lambda: fd_form(mc, torch, steps)),
             ("reuse_of_photon_tracks", lambda: rpt_form(mc, torch, steps)),
             ("coarse_grid_scatter", lambda: cgsm_form(mc, torch, steps)),
             ("tl201_dual_window", lambda: tl201_form(mc, torch, steps))]
    if not args.no_large:
        forms.append(("large_mlem", lambda: large_form(mc, torch, steps)))
    for name, run in forms:
        t = time.perf_counter()
        out[name] = run()
        # progress on stderr: the JSON line on stdout stays the only output there
        print(f"bench: form {name} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    return out


def _adjoint_step_record(mc, torch, prob, steps, rates=None):
    """Time the adjoint step on one problem: forward with an event list,
    Poisson-loss gradient against a Poisson target from an independent
    seed-1 run, replaying adjoint."""
    dp = mc.to_device(prob)
    ref = mc.simulate(dp.with_(seed=1), want_sq=False)
    lam_ref = ref.tally.view(prob.tally_shape).to(torch.float64).sum(dim=1) * 2.0 ** -32
    gen = torch.Generator(device=lam_ref.device)
    gen.manual_seed(4)
    y = torch.poisson(lam_ref, generator=gen)
    cap = max(1 << 16, 4 * int(ref.fates[0, 5].item()) + 1024)
    sim = mc.Simulator(dp, event_capacity=cap, want_sq=False)

    def loss_grad():
        lam = sim.tally.view(prob.tally_shape).to(torch.float64).sum(dim=1) * 2.0 ** -32
        eps = 1e-6 * float(prob.n_histories)
        return (1.0 - y / (lam + eps)).unsqueeze(1).expand(-1, 2, -1, -1).contiguous()

    def adjoint_step():
        sim.run()
        return mc.adjoint(dp, loss_grad(), sim)
    adjoint_step()
    ms_fwd = timed(torch, sim.run, steps)
    ms = timed(torch, adjoint_step, steps)
    timers = [mc.KernelTimer() for _ in range(steps)]
    for t in timers:
        sim.run(kernel_events=t.handles)
    torch.cuda.synchronize()
    k_fwd = float(np.mean([t.elapsed_ms() for t in timers]))
    G = loss_grad()
    ms_adj = timed(torch, lambda: mc.adjoint(dp, G, sim), steps)
    return {"value": prob.n_histories / (ms / 1e3), "unit": "histories/s",
            "ms_per_step": ms, "forward_ms": ms_fwd, "adjoint_call_ms": ms_adj,
            "histories": prob.n_histories, "tallied": int(sim.n_events.item()),
            "step": "forward with event list + Poisson-loss gradient + replaying adjoint",
            "roofline": transport_roofline(sim, k_fwd, rates)}


def adjoint_form(mc, torch, steps, rates=None):
    """Adjoint step on the 128^3 x 1 mm cube, 1e7 histories (primary), and
    on the 128^3 x 3 mm headline thorax with 60 views, 1e7 histories
    (secondary)."""
    import phantoms
    rec = _adjoint_step_record(mc, torch, phantoms.point_cube_128_adjoint(10 ** 7), steps, rates)
    rec["roofline_note"] = ("dominant kernel: the forward transport; the adjoint call replays "
                            "only the tallied histories, one wavefront each with the segment "
                            "walks split over its lanes, and reads its status back once")
    sec = _adjoint_step_record(mc, torch, phantoms.thorax_128(10 ** 7), steps, rates)
    sec["workload"] = "thorax_128: 128^3 x 3 mm thorax, 60 views, 1e7 histories"
    rec["secondary"] = sec
    return rec


def batched_form(mc, torch, steps, rates=None):
    """32 thoraxes 96^3-160^3, 30-120 views, 1e7 histories each: staging of
    every problem and one persistent transport kernel, replayed as one HIP
    graph, with the autotuned options."""
    import phantoms
    probs = phantoms.batched_thoraxes(10 ** 7)
    dps = [mc.to_device(p) for p in probs]
    opts = mc.autotune(dps, reps=1)
    s3 = mc.Simulator(dps, want_sq=False, options=opts)
    runner = mc.GraphRunner(s3)
    runner.replay()
    ms = timed(torch, runner.replay, steps)
    s3.check_status()
    timers = [mc.KernelTimer() for _ in range(steps)]
    for t in timers:
        s3.run(kernel_events=t.handles)
    torch.cuda.synchronize()
    k_ms = float(np.mean([t.elapsed_ms() for t in timers]))
    n3 = sum(p.n_histories for p in probs)
    return {"value": n3 / (ms / 1e3), "unit": "histories/s", "ms_per_step": ms,
            "transport_ms": k_ms, "histories": n3, "problems": len(probs), "options": opts,
            "launch": "hipGraph replay: staging x32 + one persistent transport kernel",
            "roofline": transport_roofline(s3, k_ms, rates)}


def fd_form(mc, torch, steps):
    """Forced detection, convolution-based forced detection, forced direction
    (into the acceptance cone) and forced interaction (Sec. 5.2) on the 128^3
    thorax, 60 views, 1e7 histories: throughput, and figures of
    merit 1 / (variance per history x time per history) against analog
    transport, for the total window count and for the projection bin by bin
    (variances summed over bins).  Analog variances are binomial, p (1 - p)
    per bin; the forced estimates' variances come from 16 independent seeds
    of 1e6 histories."""
    import phantoms
    n = 10 ** 7
    p = phantoms.thorax_128(n)
    dp = mc.to_device(p)
    sa = mc.Simulator(dp, want_sq=False)
    sa.run()
    ms_an = timed(torch, sa.run, steps)
    pb = mc.tally_float(sa.tally) / n
    p_an = float(pb.sum())
    var_an = p_an * (1.0 - p_an)
    bins_an = float((pb * (1.0 - pb)).sum())
    nz_an = int((sa.tally != 0).sum().item())
    m = 10 ** 6
    out = {}
    alpha = p.accept_half_angle_rad
    for name, opt in (("forced_detection", {"forced_detection": 1}),
                      ("convolution_fd", {"forced_detection": 2}),
                      ("forced_direction", {"variance_reduction": 1, "forced_direction_half_angle": alpha}),
                      ("forced_interaction", {"variance_reduction": 2}),
                      ("forced_direction_and_interaction",
                       {"variance_reduction": 3, "forced_direction_half_angle": alpha})):
        sf = mc.Simulator(dp, want_sq=False, options=opt)
        sf.run()
        ms = timed(torch, sf.run, steps)
        sf.check_status()
        timers = [mc.KernelTimer() for _ in range(steps)]
        for t in timers:
            sf.run(kernel_events=t.handles)
        torch.cuda.synchronize()
        k_ms = float(np.mean([t.elapsed_ms() for t in timers]))
        nz = int((sf.tally != 0).sum().item())
        kname = {"forced_detection": "k_transport_fd", "convolution_fd": "k_transport_cfd"}.get(
            name, "k_transport_vr")
        roof = forced_roofline(sf, k_ms, kname)
        del sf
        tallies = []
        for k in range(16):
            sk = mc.simulate(mc.to_device(p.with_(n_histories=m, seed=2000 + k)), want_sq=False,
                             options=opt)
            tallies.append(mc.tally_float(sk.tally) / m)
        tallies = np.stack(tallies)
        totals = tallies.sum(axis=1)
        var = float(np.var(totals, ddof=1)) * m
        bins = float(np.var(tallies, axis=0, ddof=1).sum()) * m
        t_f, t_an = ms / n, ms_an / n
        out[name] = {"value": n / (ms / 1e3), "unit": "histories/s", "ms_per_step": ms,
                     "transport_ms": k_ms, "histories": n,
                     "window_count_per_history": float(np.mean(totals)),
                     "variance_per_history": var, "bin_variance_per_history": bins,
                     "fom_gain": (var_an * t_an) / (var * t_f),
                     "bin_fom_gain": (bins_an * t_an) / (bins * t_f),
                     "nonzero_bins": nz, "roofline": roof}
    fd = out.pop("forced_detection")
    fd.update({"analog_ms_per_step": ms_an, "analog_window_count_per_history": p_an,
               "analog_variance_per_history": var_an, "analog_bin_variance_per_history": bins_an,
               "analog_nonzero_bins": nz_an, "seeds": 16})
    fd.update(out)      # the other estimators, same fields
    return fd


def rpt_form(mc, torch, steps):
    """Reuse of photon tracks (Sec. 5.3) on the 128^3 thorax, 60 views: the
    reprojection of a new estimate (each voxel of the previous one changed by
    U(-5 %, +5 %)) at 1e8 histories per previous-estimate activity, as a full
    simulation and as the previous projection plus the simulated difference
    (histories in proportion to sum |d|, the same histories per unit of
    activity)."""
    import phantoms
    p = phantoms.thorax_128(10 ** 8)
    new, prev = phantoms.estimate_pair(p.activity, 0.05, 41)
    V = p.n_views
    hpu = 1e8 / float(prev.sum(dtype=np.int64))
    a_new = float(new.sum(dtype=np.int64))
    a_diff = float(np.abs(new.astype(np.int64) - prev.astype(np.int64)).sum())
    n_full = int(round(hpu * a_new / V)) * V
    n_diff = max(1, int(round(hpu * a_diff / V))) * V
    full = mc.Simulator(mc.to_device(p.with_(activity=new, n_histories=n_full)), want_sq=False)
    diff = mc.Simulator(mc.to_device(p.with_(activity=new, activity_prev=prev, n_histories=n_diff)),
                        want_sq=False)
    full.run()
    diff.run()
    ms_full = timed(torch, full.run, steps)
    ms_diff = timed(torch, diff.run, steps)
    full.check_status()
    diff.check_status()
    neg = int((diff.tally < 0).sum().item())
    return {"full_ms": ms_full, "difference_ms": ms_diff, "histories_full": n_full,
            "histories_difference": n_diff, "difference_fraction": a_diff / a_new,
            "speedup": ms_full / ms_diff, "negative_bins": neg,
            "step": "staging + transport of the new estimate vs of the difference source"}


def cgsm_form(mc, torch, steps):
    """Coarse-grid scatter modelling (Sec. 5.4) on the 128^3 thorax, 60
    views: the forced-detection scatter projection from 1e7 histories on the
    normal problem and on the coarse one (source blocks of 2^3 voxels, 2 x 2
    pixels, expanded back), timed, and each compared (relative L2) with a
    1e8-history normal-grid reference; the history gain is the squared ratio
    of the two errors."""
    import phantoms
    n = 10 ** 7
    p = phantoms.thorax_128(n)
    dp = mc.to_device(p)
    fd = {"forced_detection": 1}
    ref = mc.simulate(dp.with_(n_histories=10 ** 8, seed=77), want_sq=False, options=fd)
    r = ref.tally.view(p.tally_shape)[:, 1].to(torch.float64) * (2.0 ** -32 / 10 ** 8)
    del ref
    fine = mc.Simulator(dp, want_sq=False, options=fd)
    cp = mc.coarse_problem(dp, 2)
    coarse = mc.Simulator(cp, want_sq=False, options=fd)

    def cgsm_step():
        coarse.run()
        return mc.expand_projection(coarse.tally, cp.tally_shape, 2)
    fine.run()
    e = cgsm_step()
    ms_fine = timed(torch, fine.run, steps)
    ms_cgsm = timed(torch, cgsm_step, steps)
    ms_coarsen = timed(torch, lambda: mc.coarse_problem(dp, 2), steps)
    f = fine.tally.view(p.tally_shape)[:, 1].to(torch.float64) * (2.0 ** -32 / n)
    c = e[:, 1] / n
    err_f = float(torch.linalg.norm(f - r) / torch.linalg.norm(r))
    err_c = float(torch.linalg.norm(c - r) / torch.linalg.norm(r))
    return {"fine_ms": ms_fine, "cgsm_ms": ms_cgsm, "coarsen_ms": ms_coarsen, "histories": n,
            "scatter_rel_l2": {"fine": err_f, "cgsm": err_c},
            "scatter_total_rel": float(c.sum() / r.sum() - 1.0),
            "history_gain": (err_f / err_c) ** 2,
            "step": "forced-detection transport of the coarse problem + expansion (coarsening "
                    "timed apart: once per source estimate)"}


def tl201_form(mc, torch, steps):
    """Tl-201 (Sec. 3) on the 128^3 thorax, 60 views: 1e8 photons split 0.9 :
    0.1 between the 71 and 167 keV lines, each acquired in both 20 %
    photopeak windows (four problems, one persistent launch; the windows of a
    line run the same photons).  value: emitted photons per second."""
    import phantoms
    base = phantoms.thorax_128(1)
    probs = phantoms.line_window_problems(base, 10 ** 8)
    dps = [mc.to_device(p) for p in probs]
    sim = mc.Simulator(dps, want_sq=False)
    sim.run()
    ms = timed(torch, sim.run, steps)
    sim.check_status()
    n_phot = sum(p.n_histories for p in probs[::2])
    fates = sim.fates.cpu().numpy()
    tal = [float(t.sum().item()) * 2.0 ** -32 for t in sim.tallies()]
    return {"value": n_phot / (ms / 1e3), "unit": "emitted photons/s", "ms_per_step": ms,
            "photons": n_phot, "histories_simulated": sum(p.n_histories for p in probs),
            "window_counts_per_photon": {
                "64-78 keV": (tal[0] + tal[2]) / n_phot, "150-184 keV": (tal[1] + tal[3]) / n_phot},
            "low_window_share_from_167_keV": tal[2] / max(tal[0] + tal[2], 1e-30),
            "photoelectric_absorbed_share_71keV": float(fates[0][0]) / probs[0].n_histories}


def large_fd(mc, torch, steps, p5):
    """Forced-detection response matrix on the large workload: 1e8 histories
    with an event list (one event per score), the weighted response matrix,
    50 MLEM iterations and 2 OSEM iterations of 8 subsets on it."""
    p = p5.with_(n_histories=10 ** 8)
    dp = mc.to_device(p)
    cap = 3 * p.n_histories
    sim = mc.Simulator(dp, event_capacity=cap, want_sq=False, options={"forced_detection": 1})
    sim.run()
    ms_fwd = timed(torch, sim.run, 1)
    n_ev = int(sim.n_events.item())
    m = mc.system_matrix(dp, sim)
    ms_sys = timed(torch, lambda: mc.system_matrix(dp, sim), 1)
    img = torch.ones(m.n_img, dtype=torch.float32, device="cuda")
    ml = mc.Mlem(m)

    def recon():
        img.fill_(1.0)
        ml.run(img, 50)
    recon()
    ms_eager = timed(torch, recon, steps)
    ms_mlem = timed(torch, mc.Graph(recon).replay, steps)

    def os_recon():
        img.fill_(1.0)
        mc.osem(m, img, 2, 8, p.nu * p.nv)
    os_recon()
    ms_os = timed(torch, os_recon, steps)
    return {"histories": p.n_histories, "forward_ms": ms_fwd, "events": n_ev,
            "events_listed": min(n_ev, cap), "system_matrix_ms": ms_sys, "nnz": m.nnz,
            "mlem_50_ms": ms_mlem, "mlem_50_eager_ms": ms_eager,
            "osem_8_subsets_2_iterations_ms": ms_os,
            "histories_per_s": p.n_histories / (ms_fwd / 1e3)}


def large_form(mc, torch, steps):
    """256^3 x 1.5 mm thorax, 120 views over 360 deg, 128^2 x 3 mm, 1e9
    histories with an event list, response matrix on the 64^3 image, 50 MLEM
    iterations, 10 OSEM iterations of 8 subsets."""
    import phantoms
    p5 = phantoms.thorax_256(10 ** 9)
    d5 = mc.to_device(p5)
    s5 = mc.Simulator(d5, event_capacity=1 << 21, want_sq=False)
    s5.run()
    ms_fwd = timed(torch, s5.run, steps)
    s5.check_status()
    m = mc.system_matrix(d5, s5)
    ms_sys = timed(torch, lambda: mc.system_matrix(d5, s5), steps)
    ml = mc.Mlem(m)
    img = torch.ones(m.n_img, dtype=torch.float32, device="cuda")

    def recon():
        img.fill_(1.0)
        ml.run(img, 50)
    recon()
    ms_eager = timed(torch, recon, steps)
    # the 50 iterations as one graph (mc_graph_begin / mc_graph_end)
    ms_mlem = timed(torch, mc.Graph(recon).replay, steps)
    # OSEM: 8 subsets of interleaved views (15 of the 120 each), 10 iterations
    img_os = torch.ones(m.n_img, dtype=torch.float32, device="cuda")

    def os_recon():
        img_os.fill_(1.0)
        mc.osem(m, img_os, 10, 8, p5.nu * p5.nv)
    os_recon()
    ms_os = timed(torch, os_recon, steps)
    n_tallied, nnz, n_bins, n_img = int(s5.n_events.item()), m.nnz, m.n_bins, m.n_img
    fd = large_fd(mc, torch, steps, p5)
    return {"value": p5.n_histories / (ms_fwd / 1e3), "unit": "histories/s",
            "forward_ms": ms_fwd, "system_matrix_ms": ms_sys, "mlem_50_ms": ms_mlem,
            "mlem_iteration_ms": ms_mlem / 50, "mlem_eager_iteration_ms": ms_eager / 50,
            "osem_8_subsets_10_iterations_ms": ms_os,
            "osem_iteration_ms": ms_os / 10, "histories": p5.n_histories,
            "tallied": n_tallied, "nnz": nnz,
            "bins": n_bins, "image_voxels": n_img, "forced_detection": fd}


if __name__ == "__main__":
    main()
