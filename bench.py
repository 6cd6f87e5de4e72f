"""Benchmark of the trapping-set search hot path on one MI355X.

Workload (one step): the (3,6)-regular PEG code N=1008, M=504 (seed 2) under
every single impulse, every pair at Tanner distance <= 4 and every tree-path
triple (about 160k patterns), searched with the int8 offset-min-sum decoder
(20 iterations) and with the float32 sum-product decoder (50 iterations), both
bisecting the impulse amplitude and sieving/deduplicating TS up to a = 12; then
importance sampling (float32 SPA, 50 iterations, 3 dB) of the four most harmful
TS found, 10^4 frames each.  Inputs are resident on the device before timing.

Prints one JSON line.  The metric is edge-updates per second (one edge x one
frame x one executed iteration), with TS found per second beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Bytes per edge-update of an edge-major streaming decoder (messages read and
# written, lambda read, APP read and written; dv = 3).  The kernels here keep
# each frame on chip, so this is an equivalence figure, not their traffic.
BYTES_PER_EU = {"oms": 3.67, "spa": 12.0}
# VALU issue peak in lane-operations: 256 CUs x 128 FP32 lanes x 2.4 GHz
# (the 157.3 TFLOP/s FP32 vector figure counts an FMA as two operations).
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# Algorithmic VALU issue slots per edge-update of each check rule: SPA = two
# phi evaluations of 3 quarter-rate transcendentals (exp2, rcp, log2; 4 slots
# each) and 5 full-rate operations, plus 6 operations for v2c, the prefix /
# suffix sums, the sign and the message rounding; OMS = 15 full-rate integer
# operations (difference, saturation, |.|, sign, min/second-min/argmin
# tracking, offset, clamp, sign application).
VALU_SLOTS_PER_EU = {"oms": 15.0, "spa": 2 * (3 * 4 + 5) + 6.0}
# HBM traffic per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled x2 and x1 by a 1 GiB copy); None once the kernel changes.
MEASURED_TRAFFIC_BYTES = {"spa": (11.93e6 + 167.06e6)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--is-frames", type=int, default=10000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--calib-copy", action="store_true",
                   help="copy 1 GiB once before timing (reference for HBM byte counters)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2208_05795_amd as tsg
    import workloads

    code = workloads.peg1008_code()
    ctx = tsg.Context(0)
    c = ctx.load_code(code)
    pats_host = c.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS, tsg.PAT_TRIPLES])
    pats = torch.from_numpy(pats_host).cuda()
    P = pats.shape[0]
    oms_kw = dict(decoder=tsg.DEC_OMS, max_iter=20, oms_offset=1, ebn0_db=3.0, k_max=512,
                  k_den=16, a_max=12)
    spa_kw = dict(decoder=tsg.DEC_SPA, max_iter=50, ebn0_db=3.0, k_max=32 * 1024, k_den=1024,
                  a_max=12)
    n_is = 4

    def step():
        rec = {}
        c.reset_ts()
        r = c.impulse_search(pats, **oms_kw)
        ts_oms = c.collect()
        rec["oms"] = r["stats"]
        c.reset_ts()
        r = c.impulse_search(pats, **spa_kw)
        ts_spa = c.collect()
        rec["spa"] = r["stats"]
        is_eu, is_ms, is_res = 0, 0.0, []
        for t in ts_spa[:n_is]:
            out = c.is_estimate(list(t.bits), 3.0, -1.0, args.is_frames, seed=7, max_iter=50)
            is_eu += out["stats"]["edge_updates"]
            is_ms += out["stats"]["decode_ms"]
            is_res.append(out)
        rec["is"] = {"edge_updates": is_eu, "decode_ms": is_ms}
        rec["ts_oms"], rec["ts_spa"], rec["is_res"] = len(ts_oms), len(ts_spa), is_res
        return rec

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    eu = sum(r["oms"]["edge_updates"] + r["spa"]["edge_updates"] + r["is"]["edge_updates"]
             for r in recs)
    ts_found = sum(r["ts_oms"] + r["ts_spa"] for r in recs)
    last = recs[-1]
    phases = {
        "oms_search": {"edge_updates": last["oms"]["edge_updates"],
                       "decode_ms": last["oms"]["decode_ms"], "sieve_ms": last["oms"]["extract_ms"],
                       "call_ms": last["oms"]["total_ms"], "ts_found": last["ts_oms"],
                       "edge_updates_per_s": last["oms"]["edge_updates"] / (last["oms"]["decode_ms"] * 1e-3)},
        "spa_search": {"edge_updates": last["spa"]["edge_updates"],
                       "decode_ms": last["spa"]["decode_ms"], "sieve_ms": last["spa"]["extract_ms"],
                       "call_ms": last["spa"]["total_ms"], "ts_found": last["ts_spa"],
                       "edge_updates_per_s": last["spa"]["edge_updates"] / (last["spa"]["decode_ms"] * 1e-3)},
        "is": {"edge_updates": last["is"]["edge_updates"], "decode_ms": last["is"]["decode_ms"],
               "frames": n_is * args.is_frames,
               "p_hat": [r["p_hat"] for r in last["is_res"]],
               "shift": [r["shift_used"] for r in last["is_res"]]},
    }
    # dominant kernel: the one with the largest time in the step
    dom = max(("oms", "spa"), key=lambda k: last[k]["decode_ms"])
    dk = last[dom]
    launch_s = dk["decode_ms"] * 1e-3 / max(dk["decode_launches"], 1)
    eu_per_launch = dk["edge_updates"] / max(dk["decode_launches"], 1)
    achieved = VALU_SLOTS_PER_EU[dom] * eu_per_launch / launch_s / 1e12
    hbm_equiv = BYTES_PER_EU[dom] * eu_per_launch / launch_s / 1e9
    roofline = {
        "bound": "alu", "kernel": f"k_search<{'SpaRule' if dom == 'spa' else 'OmsRule'}>",
        "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s",
        "frac": round(achieved / VALU_PEAK_TOPS, 4),
        "traffic": MEASURED_TRAFFIC_BYTES.get(dom),
        "per_unit": f"{VALU_SLOTS_PER_EU[dom]:g} VALU issue slots per edge-update",
        "units_per_launch": eu_per_launch,
        "launch_ms": launch_s * 1e3,
        "hbm_equivalent": {"bytes_per_edge_update": BYTES_PER_EU[dom],
                           "achieved_GBs": round(hbm_equiv, 1),
                           "frac_of_peak": round(hbm_equiv / HBM_PEAK_GBS, 4)},
    }
    line = {
        "metric": "BP edge-updates/s (TS search + IS, one job)",
        "value": eu / wall,
        "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8+f32", "data": "synthetic",
        "config": {"workload": "peg1008: (3,6) PEG N=1008 M=504, singles+pairs(d<=4)+triples, "
                               "OMS-i8 20it + SPA-f32 50it, a_max 12, 3 dB, + IS top-4 TS",
                   "patterns": int(P), "is_frames_per_ts": args.is_frames},
        "ts_found_per_s": ts_found / wall,
        "phases": phases,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(code, pats_host, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


def cpu_baseline(code, pats, seconds):
    """The oracle (plain C, OpenMP over patterns) on a bounded sample of the same
    workload: the first patterns of a fixed shuffle, OMS then SPA."""
    import numpy as np

    import oracle
    oc = oracle.OCode(code)
    rng = np.random.default_rng(0)
    order = rng.permutation(len(pats))
    threads = os.cpu_count() or 1
    eu = 0
    t_used = 0.0
    n_oms = n_spa = 0
    # OMS sample, then SPA sample, each about half of the time budget
    for dec, kw in (("oms", dict(decoder=oracle.DEC_OMS, max_iter=20, k_max=512, k_den=16)),
                    ("spa", dict(decoder=oracle.DEC_SPA, max_iter=50, k_max=32 * 1024,
                                 k_den=1024))):
        take = 256 if dec == "oms" else 16
        pos = 0
        t_phase = 0.0
        while t_phase < seconds / 2 and pos < len(pats):
            sel = np.ascontiguousarray(pats[order[pos:pos + take]])
            t0 = time.perf_counter()
            r = oracle.search(oc, sel, a_max=12, threads=threads, **kw)
            dt = time.perf_counter() - t0
            t_phase += dt
            eu += r["edge_updates"]
            pos += len(sel)
            take *= 2
        t_used += t_phase
        if dec == "oms":
            n_oms = pos
        else:
            n_spa = pos
    return {"value": eu / t_used, "unit": "edge-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_oms} OMS + {n_spa} SPA patterns of the same list (fixed shuffle), "
                      f"{t_used:.1f} s"}


if __name__ == "__main__":
    main()
