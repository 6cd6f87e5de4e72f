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
# algorithmic bytes per edge-update of the edge-major streaming formulation
# (messages read + written, lambda read, APP read + written; dv = 3)
BYTES_PER_EU = {"oms": 3.67, "spa": 12.0}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--is-frames", type=int, default=10000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
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
    achieved = BYTES_PER_EU[dom] * dk["edge_updates"] / (dk["decode_ms"] * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": f"k_search_{dom}",
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "bytes_per_edge_update": BYTES_PER_EU[dom],
        "launch_ms": dk["decode_ms"] / max(dk["decode_launches"], 1),
        "launches": dk["decode_launches"],
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
