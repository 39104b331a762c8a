"""Region profile of the transport loop on the 128^3 thorax headline workload.

Loads the measurement build (libmcspect_prof.so: the library's sources with
the MC_REGION markers compiled in), runs one untimed and one profiled
simulate call, and prints one JSON record: for every region of the loop the
number of wave-level entries (exact), entries per wave iteration, and its
share of the wave-clock time (the markers themselves cost about as much as a
short region; the share of RG_LOOP, whose region holds almost no code, shows
that cost).

    python paper_2105_13324_amd/region_profile.py [--histories 1e8]

(run as a script: importing the package first would load the product library)
"""
import argparse
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

REGIONS = ["loop", "refill", "emit", "begin_history", "exit_test", "philox", "step", "escape", "gather",
           "kahn", "kahn_accept", "accept_test", "real_collision", "energy_terms", "fate_energy",
           "work_count", "fates", "tally", "forced", "before_first_marker"]


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--histories", type=float, default=1e8)
    args = ap.parse_args()
    prof = os.path.join(HERE, "libmcspect_prof.so")
    if not os.path.exists(prof):
        raise SystemExit("libmcspect_prof.so is not built: run python paper_2105_13324_amd/build.py --profile")
    os.environ["MCSPECT_LIB"] = prof
    sys.path.insert(0, ROOT)
    import torch
    import paper_2105_13324_amd as mc
    import phantoms
    lib = mc._lib
    lib.mc_region_profile.argtypes = [C.POINTER(C.c_ulonglong), C.POINTER(C.c_ulonglong), C.c_int]
    n = len(REGIONS)
    cnt, cyc = (C.c_ulonglong * n)(), (C.c_ulonglong * n)()
    prob = phantoms.thorax_128(int(args.histories))
    sim = mc.Simulator(mc.to_device(prob), want_sq=True)
    sim.run()
    torch.cuda.synchronize()
    if lib.mc_region_profile(cnt, cyc, 1) != 0:
        raise RuntimeError("mc_region_profile reset failed")
    sim.run()
    torch.cuda.synchronize()
    if lib.mc_region_profile(cnt, cyc, 0) != 0:
        raise RuntimeError("mc_region_profile read failed")
    sim.check_status()
    iters = cnt[0]
    total = sum(cyc)
    per = sim.counters.cpu().numpy()[0]
    rec = {"workload": "thorax_128", "histories": int(args.histories), "wave_iterations": int(iters),
           "lane_iterations_per_wave_iteration": float((per[0] + per[2]) / max(iters, 1)),
           "regions": {r: {"entries": int(cnt[i]), "per_iteration": cnt[i] / max(iters, 1),
                           "time_share": cyc[i] / max(total, 1)} for i, r in enumerate(REGIONS)}}
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
