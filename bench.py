"""Benchmark of the trapping-set search hot path on one MI355X.

Workload (one step): the (3,6)-regular PEG code N=1008, M=504 (seed 2) under
every single impulse, every pair at Tanner distance <= 4 and every tree-path
triple (about 160k patterns), searched with the int8 offset-min-sum decoder
(20 iterations) and with the float32 sum-product decoder (50 iterations), both
bisecting the impulse amplitude and sieving/deduplicating TS up to a = 12; then
importance sampling (float32 SPA, 50 iterations, 3 dB) of the four most harmful
TS found, 10^4 frames each.  Inputs are resident on the device before timing.

Beside it, with their own figures in the same JSON line:
  batched  - 64 QC codes of uneven size (bases 3x6/4x8/3x12/4x24, Z 16..384,
             N 96..9216), each with 4096 impulse patterns (OMS-i8, 20 it.) and
             16384 IS frames (SPA with Q20 messages and f32 phi, 50 it., 3 dB, s = 1 on the shortest cycle
             through variable 0): every job alone versus all 128 in one batch
             (ts_run_batch), results checked identical;
  served   - a Poisson stream (20 jobs/s) of search and IS jobs on 46x68-base QC
             codes (N up to 25.7k), 10^3..10^5 frames each (log-uniform),
             through ts_submit: p50/p99 latency and edge-updates/s;
  qc2640   - the (2640,1320) girth-8 QC stand-in: every tree-path triple
             searched with SPA, and one triple per orbit of the circulant shift
             (same TS); then the union bound over the (up to) 16 most harmful TS at
             2/3/4/5 dB, 10^5 IS frames each.

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
MEASURED_TRAFFIC_BYTES = {"spa": (30.24e6 + 118.07e6)}
# Same for the streamed-layout launch of the QC-2640 triples search (qc2640
# section); None until measured on the current kernel.
MEASURED_STREAMED_TRAFFIC_BYTES = 239161.94e6 + 708311.64e6


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
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--no-qc2640", action="store_true")
    p.add_argument("--no-layered", action="store_true")
    p.add_argument("--only", choices=["batch", "serve", "qc2640", "layered"],
                   help="run only this section (profiling aid); prints its JSON object")
    p.add_argument("--serve-seconds", type=float, default=60.0)
    p.add_argument("--serve-capacity-jobs", type=int, default=300,
                   help="jobs of the stream rerun all at once and through the plain calls")
    p.add_argument("--serve-rate", type=float, default=20.0)
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2208_05795_amd as tsg
    import workloads

    if args.calib_copy:
        calib_copy(torch)
    if args.only:
        fn = {"batch": lambda: bench_batch(tsg),
              "serve": lambda: bench_serve(tsg, args.serve_seconds, args.serve_rate,
                                           capacity_jobs=args.serve_capacity_jobs),
              "qc2640": lambda: bench_qc2640(tsg),
              "layered": lambda: bench_layered(tsg)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return

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
        ts_oms, _ = c.collect_arrays()   # the TS table as arrays (no per-set objects)
        rec["oms"] = r["stats"]
        c.reset_ts()
        r = c.impulse_search(pats, **spa_kw)
        ts_spa, spa_bits = c.collect_arrays()
        rec["spa"] = r["stats"]
        rec["spa_out"] = {k: r[k] for k in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")}
        # IS of the most harmful sets as one batch (their eps* shifts from one
        # search launch, their frames in one persistent launch)
        jobs = [("is", c, spa_bits[t["bits_off"]:t["bits_off"] + t["a"]],
                 dict(ebn0_db=3.0, shift=-1.0, n_frames=args.is_frames, seed=7, max_iter=50))
                for t in ts_spa[:n_is]]
        ids = ctx.run_batch(jobs)
        st = ctx.stats()
        infos = [ctx.poll(j) for j in ids]
        for j in ids:
            ctx.release(j)
        is_res = [i["is"] for i in infos]
        rec["is"] = {"edge_updates": sum(i["edge_updates"] for i in infos), "decode_ms": st["decode_ms"]}
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
    # outside the timed steps: the same SPA search with every iteration of every
    # decode computed (no fixed-point exit), for the kernel's rate on full decodes
    c.reset_ts()
    rf = c.impulse_search(pats, full_iterations=True, **spa_kw)
    ts_full = c.collect()
    full = rf["stats"]
    full_same = (len(ts_full) == recs[-1]["ts_spa"] and
                 all(torch.equal(rf[k], v) for k, v in recs[-1]["spa_out"].items()))
    # and the step's IS batch likewise (the oracle computes every iteration)
    ids = ctx.run_batch([("is", c, list(t.bits), dict(ebn0_db=3.0, shift=-1.0, n_frames=args.is_frames,
                                                       seed=7, max_iter=50, full_iterations=True))
                         for t in ts_full[:n_is]])
    is_full_eu = sum(ctx.poll(j)["edge_updates"] for j in ids)
    for j in ids:
        ctx.release(j)
    ts_found = sum(r["ts_oms"] + r["ts_spa"] for r in recs)
    cands = sum(r["oms"]["candidates"] + r["spa"]["candidates"] for r in recs)
    lds_peak = ctx.probe_lds()
    last = recs[-1]
    phases = {
        "oms_search": {"edge_updates": last["oms"]["edge_updates"],
                       "decode_ms": last["oms"]["decode_ms"], "sieve_ms": last["oms"]["extract_ms"],
                       "call_ms": last["oms"]["total_ms"], "ts_found": last["ts_oms"],
                       "edge_updates_per_s": last["oms"]["edge_updates"] / (last["oms"]["decode_ms"] * 1e-3)},
        "spa_search": {"edge_updates": last["spa"]["edge_updates"],
                       "decode_ms": last["spa"]["decode_ms"], "sieve_ms": last["spa"]["extract_ms"],
                       "call_ms": last["spa"]["total_ms"], "ts_found": last["ts_spa"],
                       "edge_updates_per_s": last["spa"]["edge_updates"] / (last["spa"]["decode_ms"] * 1e-3),
                       "shape": {k: last["spa"][k] for k in ("layout", "block_threads", "checks_per_thread",
                                                              "grid_blocks")}},
        "spa_search_full_iterations": {
            "edge_updates": full["edge_updates"], "decode_ms": full["decode_ms"],
            "edge_updates_per_s": full["edge_updates"] / (full["decode_ms"] * 1e-3),
            "same_results": bool(full_same)},
        "is": {"edge_updates": last["is"]["edge_updates"], "decode_ms": last["is"]["decode_ms"],
               "edge_updates_full_iterations": is_full_eu,
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
    # LDS bytes per edge-update of the register layout: the APP gather (4) and
    # the atomic add (read + write, 8) per edge, and per variable the channel
    # read, the next APP buffer's initialisation and the hard-decision read
    # (12) spread over its edges
    lds_bpe = 12.0 + 12.0 * code.n / c.e
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
        "lds": {"bytes_per_edge_update": round(lds_bpe, 3),
                "achieved_GBs": round(lds_bpe * eu_per_launch / launch_s / 1e9, 1),
                "peak_GBs_measured": round(lds_peak / 1e9, 1),
                "frac_of_measured_peak": round(lds_bpe * eu_per_launch / launch_s / lds_peak, 4)},
        # the same kernel on the same patterns with every iteration computed
        "full_iterations_frac": round(VALU_SLOTS_PER_EU["spa"] * full["edge_updates"]
                                      / (full["decode_ms"] * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
    }
    line = {
        "metric": "BP edge-updates/s (TS search + IS, one job)",
        "value": eu / wall,
        "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8+q20/f32", "data": "synthetic",
        "config": {"workload": "peg1008: (3,6) PEG N=1008 M=504, singles+pairs(d<=4)+triples, "
                               "OMS-i8 20it + SPA-q20/f32 50it, a_max 12, 3 dB, + IS top-4 TS",
                   "patterns": int(P), "is_frames_per_ts": args.is_frames},
        "ts_found_per_s": ts_found / wall,
        "candidates_per_s": cands / wall,
        "phases": phases,
        "roofline": roofline,
    }
    ctx.close()
    del pats
    if not args.no_batch:
        line["batched"] = bench_batch(tsg)
    if not args.no_serve:
        line["served"] = bench_serve(tsg, args.serve_seconds, args.serve_rate,
                                     capacity_jobs=args.serve_capacity_jobs)
    if not args.no_qc2640:
        line["qc2640"] = bench_qc2640(tsg)
    if not args.no_layered:
        line["layered"] = bench_layered(tsg)
    if not args.no_cpu_baseline:
        # the oracle computes every iteration: its share of each leg is the
        # full-iteration edge-updates; the rate is quoted in the step's
        # computed edge-updates, so that GPU / CPU is the ratio of the times
        mix = {"oms": last["oms"]["edge_updates"], "spa": full["edge_updates"], "is": is_full_eu}
        step_eu = last["oms"]["edge_updates"] + last["spa"]["edge_updates"] + last["is"]["edge_updates"]
        line["cpu_baseline"] = cpu_baseline(code, pats_host, args.cpu_seconds, mix, step_eu)
    print(json.dumps(line), flush=True)


def _say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def calib_copy(torch):
    """One 1 GiB device-to-device copy: the byte reference of the HBM counters."""
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def var_checks(rp, col, n):
    """Checks of every variable, from the check-major CSR."""
    import numpy as np
    m = len(rp) - 1
    rows = np.repeat(np.arange(m), np.diff(rp))
    order = np.argsort(col, kind="stable")
    vptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(vptr, col.astype(np.int64) + 1, 1)
    return np.cumsum(vptr), rows[order]


def shortest_cycle_vns(graph, v0):
    """Variables of a shortest Tanner-graph cycle through variable v0 (BFS with
    one branch label per neighbouring check of v0).  graph = (rp, col, vptr,
    vchk, n)."""
    rp, col, vptr, vchk, n = graph
    parent = {v0: -1}
    branch = {v0: -1}
    dist = {v0: 0}
    frontier = [v0]
    best = None
    while frontier and best is None:
        nxt = []
        for u in frontier:
            if u < n:
                nbrs = [int(c) + n for c in vchk[vptr[u]:vptr[u + 1]]]
            else:
                nbrs = [int(v) for v in col[rp[u - n]:rp[u - n + 1]]]
            for w in nbrs:
                if w == parent[u]:
                    continue
                if w in dist:
                    if branch[w] != branch[u] and w != v0 and u != v0:
                        L = dist[u] + dist[w] + 1
                        if best is None or L < best[0]:
                            best = (L, u, w)
                    continue
                dist[w] = dist[u] + 1
                parent[w] = u
                branch[w] = w if u == v0 else branch[u]
                nxt.append(w)
        frontier = nxt
    if best is None:
        return [v0]
    _, u, w = best
    vs = set()
    for x in (u, w):
        while x != -1:
            if x < n:
                vs.add(x)
            x = parent[x]
    return sorted(vs)


def sample_pairs(graph, count, rng):
    """count impulse pairs (u, w) at Tanner distance 2: u uniform, then one of its
    checks, then another variable of that check."""
    import numpy as np
    rp, col, vptr, vchk, n = graph
    u = rng.integers(0, n, size=count)
    deg_u = vptr[u + 1] - vptr[u]
    c = vchk[vptr[u] + (rng.random(count) * deg_u).astype(np.int64)]
    deg_c = rp[c + 1] - rp[c]
    k = (rng.random(count) * deg_c).astype(np.int64)
    w = col[rp[c] + k]
    w = np.where(w == u, col[rp[c] + (k + 1) % deg_c], w)   # the next variable of the check
    out = np.stack([np.minimum(u, w), np.maximum(u, w)], axis=1).astype(np.int32)
    return np.ascontiguousarray(out)


def _job_results(ctx, ids, jobs):
    out = []
    for (kind, _, _, _), jid in zip(jobs, ids):
        info = ctx.poll(jid, wait=True)
        if info["status"] != 0:
            raise RuntimeError(f"job {jid} failed: {info.get('error')}")
        if kind == "search":
            o = ctx.job_outputs(jid, arrays=True)
            out.append(("search", o["k_crit"], (o["ts_recs"], o["ts_bits"]), info["edge_updates"]))
        else:
            out.append(("is", info["is"]["p_hat"], info["is"]["n_fail"], info["edge_updates"]))
        ctx.release(jid)
    return out


def bench_batch(tsg):
    """64 uneven QC codes: every job alone, then all of them as one batch, three
    alternating times after a warm-up of each; the medians are reported."""
    import numpy as np
    import workloads
    codes = workloads.batch_codes()
    rng = np.random.default_rng(4)
    ctx = tsg.Context(0)
    loaded = [ctx.load_code(c) for c in codes]
    jobs = []
    for i, (c, g) in enumerate(zip(codes, loaded)):
        pats = np.full((4096, 2), -1, dtype=np.int32)
        k = min(c.n, 4096)
        pats[:k, 0] = np.arange(k)
        if k < 4096:
            pairs = g.make_patterns(tsg.PAT_PAIRS)
            sel = np.sort(rng.choice(len(pairs), 4096 - k, replace=False))
            pats[k:] = pairs[sel]
        rp, col = g.csr()
        bits = shortest_cycle_vns((rp, col) + var_checks(rp, col, c.n) + (c.n,), 0)
        jobs.append(("search", g, pats, dict(a_max=12)))
        jobs.append(("is", g, bits, dict(ebn0_db=3.0, shift=1.0, n_frames=16384, seed=40 + i,
                                         max_iter=50)))

    def plain(jobs):
        res = []
        for kind, g, data, kw in jobs:
            if kind == "search":
                g.reset_ts()
                r = g.impulse_search(data, **kw)
                res.append(("search", r["k_crit"], g.collect_arrays(), r["stats"]["edge_updates"]))
            else:
                kw = dict(kw)
                r = g.is_estimate(data, kw.pop("ebn0_db"), kw.pop("shift"), kw.pop("n_frames"),
                                  kw.pop("seed"), **kw)
                res.append(("is", r["p_hat"], r["n_fail"], r["stats"]["edge_updates"]))
        return res

    def batched(jobs):
        ids = ctx.run_batch(jobs)
        st = ctx.stats()
        return _job_results(ctx, ids, jobs), st

    def timed_pairs(js, reps):
        """reps alternating runs of each form; the medians and every time."""
        tp, tb, same = [], [], True
        for _ in range(reps):
            t0 = time.perf_counter()
            ref = plain(js)
            tp.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            got, st = batched(js)
            tb.append(time.perf_counter() - t0)
            same = same and all(same_job(a, b) for a, b in zip(ref, got))
        return float(np.median(tp)), float(np.median(tb)), tp, tb, ref, st, same

    def same_job(a, b):
        if a[0] != b[0] or a[3] != b[3]:
            return False
        if a[0] == "is":
            return a[1] == b[1] and a[2] == b[2]
        return (np.array_equal(a[1], b[1]) and np.array_equal(a[2][0], b[2][0])
                and np.array_equal(a[2][1], b[2][1]))
    _say("batched: warm-up (autotunes every code)")
    plain(jobs)
    batched(jobs)
    t_plain, t_batch, tps, tbs, ref, st, same = timed_pairs(jobs, 3)
    eu = sum(r[3] for r in ref)
    ts = sum(len(r[2][0]) for r in ref if r[0] == "search")
    # the same codes with small jobs (256 patterns, 1024 IS frames): a plain
    # call no longer fills the device, a batch still does
    small = []
    for kind, g, data, kw in jobs:
        if kind == "search":
            small.append((kind, g, np.ascontiguousarray(data[:256]), kw))
        else:
            small.append((kind, g, data, dict(kw, n_frames=1024)))
    plain(small)
    batched(small)
    t_plain_s, t_batch_s, tps_s, tbs_s, ref_s, _, same_s = timed_pairs(small, 3)
    eu_s = sum(r[3] for r in ref_s)
    ctx.close()
    return {"workload": "64 QC codes, bases 3x6/4x8/3x12/4x24, Z 16..384 (seed 4); per code 4096 "
                        "impulse patterns OMS-i8 20it + 16384 IS frames SPA (Q20 messages, f32 phi) 50it at 3 dB",
            "jobs": len(jobs), "edge_updates": eu, "ts_found": ts,
            "plain": {"seconds": t_plain, "edge_updates_per_s": eu / t_plain,
                      "ts_found_per_s": ts / t_plain},
            "batched": {"seconds": t_batch, "edge_updates_per_s": eu / t_batch,
                        "ts_found_per_s": ts / t_batch, "decode_launches": st["decode_launches"]},
            "speedup": t_plain / t_batch, "results_identical": bool(same),
            "timing": "median of 3 alternating runs of each form",
            "plain_runs_s": tps, "batched_runs_s": tbs,
            "small_jobs": {"workload": "the same 64 codes, 256 patterns + 1024 IS frames per code",
                           "plain_s": t_plain_s, "batched_s": t_batch_s,
                           "plain_runs_s": tps_s, "batched_runs_s": tbs_s,
                           "plain_edge_updates_per_s": eu_s / t_plain_s,
                           "batched_edge_updates_per_s": eu_s / t_batch_s,
                           "speedup": t_plain_s / t_batch_s, "results_identical": bool(same_s)}}


def _serve_stream(pool, graphs, rng, seconds, rate):
    """Poisson arrivals over [0, seconds): (arrival, kind, code index, data, kwargs)."""
    t, jobs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        ci = int(rng.integers(0, len(pool)))
        frames = int(round(10 ** rng.uniform(3, 5)))
        c = pool[ci]
        if rng.random() < 0.5:
            jobs.append((t, "search", ci, sample_pairs(graphs[ci], frames, rng), dict(a_max=12)))
        else:
            v0 = int(rng.integers(0, c.n))
            bits = shortest_cycle_vns(graphs[ci], v0)[:16]
            jobs.append((t, "is", ci, bits, dict(ebn0_db=float(rng.integers(2, 6)), shift=1.0,
                                                 n_frames=frames, seed=int(rng.integers(1 << 30)),
                                                 max_iter=50)))
    return jobs


def _warm(loaded, graphs, jobs):
    """Runs one small search and one small IS estimate per code the jobs use,
    so that the autotuner's probes (cached per code) fall outside the timing."""
    import numpy as np
    rng = np.random.default_rng(9)
    skw = next(j[4] for j in jobs if j[1] == "search")
    for ci in sorted({j[2] for j in jobs}):
        g = loaded[ci]
        # sizes at which a plain call tunes (256 patterns, 1024 frames)
        g.impulse_search(sample_pairs(graphs[ci], 512, rng), **skw)
        g.reset_ts()
        g.is_estimate(shortest_cycle_vns(graphs[ci], 0)[:16], 3.0, 1.0, 2048, seed=1, max_iter=50)


def _serve_run(tsg, pool, graphs, jobs, budget, paced):
    """Runs the jobs through the serving loop (4 worker slots) on a fresh
    context; paced = submit at the arrival times, else all at once."""
    import numpy as np
    ctx = tsg.Context(0, torch_stream=False, torch_alloc=False, hbm_budget_bytes=budget)
    loaded = [ctx.load_code(c) for c in pool]
    _warm(loaded, graphs, jobs)
    ctx.serve_start(4)
    ids = []
    t0 = time.perf_counter()
    for ta, kind, ci, data, kw in jobs:
        now = time.perf_counter() - t0
        if paced and ta > now:
            time.sleep(ta - now)
        g = loaded[ci]
        if kind == "search":
            ids.append(ctx.submit_search(g, data, **kw))
        else:
            kw = dict(kw)
            ids.append(ctx.submit_is(g, data, kw.pop("ebn0_db"), kw.pop("shift"), kw.pop("n_frames"),
                                     kw.pop("seed"), **kw))
    infos = [ctx.poll(j, wait=True) for j in ids]
    wall = time.perf_counter() - t0
    for j in ids:
        ctx.release(j)
    ctx.close()
    lat = np.array([i["end_ms"] - i["submit_ms"] for i in infos])
    eu = sum(i["edge_updates"] for i in infos)
    span = (max(i["end_ms"] for i in infos) - min(i["submit_ms"] for i in infos)) * 1e-3
    return {"jobs": len(ids), "failed": sum(1 for i in infos if i["status"] != 0),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "edge_updates": int(eu), "edge_updates_per_s": eu / span, "seconds": span, "wall_s": wall}


def _plain_run(tsg, pool, graphs, jobs):
    """The same jobs one after another through the plain per-job calls."""
    import numpy as np
    ctx = tsg.Context(0, torch_stream=False, torch_alloc=False)
    loaded = [ctx.load_code(c) for c in pool]
    _warm(loaded, graphs, jobs)
    eu = 0
    t0 = time.perf_counter()
    for _, kind, ci, data, kw in jobs:
        g = loaded[ci]
        if kind == "search":
            g.reset_ts()
            r = g.impulse_search(data, **kw)
            g.collect_arrays()
        else:
            kw = dict(kw)
            r = g.is_estimate(data, kw.pop("ebn0_db"), kw.pop("shift"), kw.pop("n_frames"),
                              kw.pop("seed"), **kw)
        eu += r["stats"]["edge_updates"]
    wall = time.perf_counter() - t0
    ctx.close()
    return {"edge_updates": int(eu), "seconds": wall, "edge_updates_per_s": eu / wall}


def bench_serve(tsg, seconds, rate, stress_seconds=5.0, capacity_jobs=300):
    """Poisson arrivals of search and IS jobs on the 46x68-base code pool:
    the paced stream under a 32 GiB HBM budget (latency), the stream's first
    capacity_jobs jobs all submitted at once (capacity) and one after another
    through the plain per-job calls, and a short paced stream under a 1 GiB
    budget (admission stress)."""
    import numpy as np
    import workloads
    pool = workloads.serving_pool()
    rng = np.random.default_rng(5)
    graphs = []
    ctx = tsg.Context(0, torch_stream=False, torch_alloc=False)
    for c in pool:   # the expanded graphs, from the library's loader
        g = ctx.load_code(c)
        rp, col = g.csr()
        graphs.append((rp, col) + var_checks(rp, col, c.n) + (c.n,))
    ctx.close()
    jobs = _serve_stream(pool, graphs, rng, seconds, rate)
    _say(f"served: {len(jobs)} jobs paced over {seconds:.0f} s")
    paced = _serve_run(tsg, pool, graphs, jobs, 32 << 30, True)
    cap = jobs[:capacity_jobs]
    _say(f"served: the first {len(cap)} jobs submitted at once")
    burst = _serve_run(tsg, pool, graphs, cap, 32 << 30, False)
    _say("plain: the same jobs one after another")
    plain = _plain_run(tsg, pool, graphs, cap)
    stress_jobs = _serve_stream(pool, graphs, np.random.default_rng(55), stress_seconds, rate)
    _say(f"served: {len(stress_jobs)} jobs paced over {stress_seconds:.0f} s under a 1 GiB budget")
    stress = _serve_run(tsg, pool, graphs, stress_jobs, 1 << 30, True)
    out = {"workload": f"Poisson {rate:g} jobs/s for {seconds:g} s, 46x68-base QC pool of 32 "
                       "(N up to 25.7k), 50/50 search (OMS-i8 20it) / IS (SPA-q20/f32 50it, 2..5 dB), "
                       "10^3..10^5 frames log-uniform, 4 worker slots, 32 GiB HBM budget"}
    out.update(paced)
    out["all_at_once"] = dict(burst, jobs_of_stream=len(cap))
    out["plain_sequential"] = plain
    out["served_vs_plain"] = burst["edge_updates_per_s"] / plain["edge_updates_per_s"]
    out["stress_1GiB"] = stress
    return out


def bench_qc2640(tsg):
    """QC-2640: SPA search over every tree-path triple and over one triple per
    orbit of the circulant shift (same TS), then the union bound over the (up to) 16
    most harmful TS at 2, 3, 4, 5 dB with 10^5 IS frames each (shift eps*)."""
    import numpy as np
    import workloads
    ctx = tsg.Context(0)
    g = ctx.load_code(workloads.qc2640_code())
    pats = g.make_patterns(tsg.PAT_TRIPLES)
    reps = g.make_patterns(tsg.PAT_TRIPLES | tsg.PAT_QC_ORBITS)
    kw = dict(decoder=tsg.DEC_SPA, max_iter=50, ebn0_db=3.0, k_max=32 * 1024, k_den=1024, a_max=12)
    g.impulse_search(pats[:4096], **kw)   # warm-up / autotune
    g.impulse_search(reps, **kw)
    g.reset_ts()
    t0 = time.perf_counter()
    r = g.impulse_search(pats, **kw)
    recs, _ = g.collect_arrays()
    t_search = time.perf_counter() - t0
    eu_search = r["stats"]["edge_updates"]
    g.reset_ts()
    t0 = time.perf_counter()
    rr = g.impulse_search(reps, **kw)
    recs_r, _ = g.collect_arrays()
    t_reduced = time.perf_counter() - t0
    same = bool(np.array_equal(recs[["a", "b", "orbit", "k_crit"]], recs_r[["a", "b", "orbit", "k_crit"]]))
    spectrum = g.spectrum(a_max=12, b_max=12, by_orbit=False)
    # the same search in the streamed layout (messages through global memory),
    # the form the edge-major roofline describes
    g.reset_ts()
    rs = g.impulse_search(pats, layout=tsg.LAYOUT_STREAMED, **kw)
    recs_s, _ = g.collect_arrays()
    st_s = rs["stats"]
    same_s = bool(np.array_equal(recs, recs_s))
    n_ts = min(16, len(recs_r))
    snrs = [2.0, 3.0, 4.0, 5.0]
    t0 = time.perf_counter()
    ub = g.union_bound(n_ts, snrs, 100000, seed=3, shift=-1.0, per_ts=True,
                       count_mode=tsg.IS_COUNT_TS, shift_rule=tsg.SHIFT_MIX)
    t_ub = time.perf_counter() - t0
    eu_ub = ub["stats"]["edge_updates"]
    ctx.close()
    launch_s = st_s["decode_ms"] * 1e-3 / max(st_s["decode_launches"], 1)
    eu_launch = st_s["edge_updates"] / max(st_s["decode_launches"], 1)
    ach = BYTES_PER_EU["spa"] * eu_launch / launch_s / 1e9
    roof_s = {"bound": "hbm", "kernel": "k_search_g<SpaRule>", "unit": "GB/s",
              "bytes_per_edge_update": BYTES_PER_EU["spa"], "units_per_launch": eu_launch,
              "launch_ms": launch_s * 1e3, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
              "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": MEASURED_STREAMED_TRAFFIC_BYTES,
              "variant": "accumulating" if st_s["checks_per_thread"] else "gathering",
              "grid_blocks": st_s["grid_blocks"], "block_threads": st_s["block_threads"],
              "same_ts": same_s}
    cells = {f"{a},{b}": int(spectrum[a, b]) for a in range(spectrum.shape[0])
             for b in range(spectrum.shape[1]) if spectrum[a, b]}
    return {"workload": "QC (3,6) N=2640 Z=440 girth 8 (seed 3): SPA-q20/f32 50it search over "
                        f"{len(pats)} triples and over the {len(reps)} orbit representatives, then the "
                        f"union bound over the top {n_ts} TS x 4 SNRs x 1e5 IS frames",
            "ts_found": int(len(recs)), "spectrum_all_sets": cells,
            "search": {"seconds": t_search, "edge_updates": eu_search,
                       "edge_updates_per_s": eu_search / t_search,
                       "hbm_equivalent_frac": BYTES_PER_EU["spa"] * eu_search / t_search / (HBM_PEAK_GBS * 1e9)},
            "roofline_streamed": roof_s,
            "search_orbit_reduced": {"patterns": int(len(reps)), "seconds": t_reduced,
                                     "edge_updates": rr["stats"]["edge_updates"],
                                     "speedup": t_search / t_reduced, "same_ts": same},
            "union_bound": {"seconds": t_ub, "edge_updates": eu_ub, "edge_updates_per_s": eu_ub / t_ub,
                            "fer": {f"{p['ebn0_db']:g}dB": {"fer": p["fer"], "ci": [p["ci_lo"], p["ci_hi"]]}
                                    for p in ub["points"]},
                            "estimator": "frames split over the shifts eps* k/16, k = 0..16, "
                                         "balance-heuristic weights; counts the set's own error events",
                            # per SNR, per set of the table: (shift, counted frames, P_hat, CI)
                            "per_ts": {f"{p['ebn0_db']:g}dB": [[r["shift_used"], r["n_fail"], r["p_hat"],
                                                                [r["ci_lo"], r["ci_hi"]]]
                                                               for r in rows]
                                       for p, rows in zip(ub["points"], ub["per_ts"])}}}


def bench_layered(tsg):
    """The quantised normalised layered min-sum (4/4/6 bits, 20 iterations, the
    decoder of Fig. 2) as the impulse-search decoder: the whole PEG-1008 list
    (greedy layers) and every QC-2640 triple (block-row layers), at 3 dB with
    the channel at full scale and at 0.3 x scale (where impulses fail)."""
    import workloads
    out = {}
    for name, fn, kinds in (("peg1008", workloads.peg1008_code,
                             [tsg.PAT_SINGLES, tsg.PAT_PAIRS, tsg.PAT_TRIPLES]),
                            ("qc2640", workloads.qc2640_code, [tsg.PAT_TRIPLES])):
        ctx = tsg.Context(0)
        g = ctx.load_code(fn())
        pats = g.pattern_list(kinds)
        for scale in (1.0, 0.3):
            kw = dict(decoder=tsg.DEC_LNMS, max_iter=20, ebn0_db=3.0, llr_scale=scale, k_max=512,
                      k_den=16, a_max=12)
            g.impulse_search(pats[:4096], **kw)   # warm-up / autotune
            g.reset_ts()
            t0 = time.perf_counter()
            r = g.impulse_search(pats, **kw)
            recs, _ = g.collect_arrays()
            dt = time.perf_counter() - t0
            st = r["stats"]
            out[f"{name}_x{scale:g}"] = {
                "patterns": int(len(pats)), "layers": int(g.info["n_layers"]),
                "seconds": dt, "edge_updates": st["edge_updates"],
                "edge_updates_per_s": st["edge_updates"] / dt,
                "kernel_edge_updates_per_s": st["edge_updates"] / (st["decode_ms"] * 1e-3),
                "failing_patterns": int((r["k_crit"] >= 0).sum()), "ts_found": int(len(recs)),
                "shape": {"layout": st["layout"], "checks_per_thread": st["checks_per_thread"]}}
        ctx.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(code, pats, seconds, mix, step_eu):
    """The oracle (plain C, OpenMP over patterns / frames) on bounded samples of
    the same workload, on all host threads: OMS and SPA searches over the first
    patterns of a fixed shuffle, and IS frames (SPA, 3 dB, shift 1.5) of the
    shortest cycle through variable 0.  The oracle's time for the step is the
    sum over legs of the leg's full-iteration edge-updates (mix) over the
    oracle's rate on that leg; the reported rate is the step's computed
    edge-updates (step_eu) over that time.  A single-thread SPA sample is
    reported beside it."""
    import numpy as np

    import oracle
    import workloads
    oc = oracle.OCode(code)
    rng = np.random.default_rng(0)
    order = rng.permutation(len(pats))
    threads = os.cpu_count() or 1
    legs = {}

    def search_leg(kw, take, budget, nthreads):
        pos, t_used, eu = 0, 0.0, 0
        while t_used < budget and pos < len(pats):
            sel = np.ascontiguousarray(pats[order[pos:pos + take]])
            t0 = time.perf_counter()
            r = oracle.search(oc, sel, a_max=12, threads=nthreads, **kw)
            t_used += time.perf_counter() - t0
            eu += r["edge_updates"]
            pos += len(sel)
            take *= 2
        return {"patterns": pos, "seconds": t_used, "edge_updates_per_s": eu / t_used}

    legs["oms"] = search_leg(dict(decoder=oracle.DEC_OMS, max_iter=20, k_max=512, k_den=16),
                             256, 0.25 * seconds, threads)
    # the oracle spreads patterns over its threads in chunks: give each thread several
    legs["spa"] = search_leg(dict(decoder=oracle.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024),
                             8 * threads, 0.35 * seconds, threads)
    rp, col = oc.csr()
    graph = (rp, col) + var_checks(rp, col, code.n) + (code.n,)
    bits = shortest_cycle_vns(graph, 0)
    frames, t_used, eu = 256, 0.0, 0
    n_frames = 0
    while t_used < 0.2 * seconds:
        t0 = time.perf_counter()
        r = oracle.is_estimate(oc, bits, 3.0, 1.5, frames, seed=7, frame_base=n_frames,
                               threads=threads)
        t_used += time.perf_counter() - t0
        eu += r["edge_updates"]
        n_frames += frames
        frames *= 2
    legs["is"] = {"frames": n_frames, "seconds": t_used, "edge_updates_per_s": eu / t_used}
    # beside the mix: IS frames on the QC-2640 code (its shortest cycle through
    # variable 0, 3 dB, shift 1.5), a counter-addressed subset of the same
    # Philox frames the device draws
    qc = workloads.qc2640_code()
    oq = oracle.OCode(qc)
    rq, cq = oq.csr()
    qbits = shortest_cycle_vns((rq, cq) + var_checks(rq, cq, qc.n) + (qc.n,), 0)
    frames, t_q, eu_q, nq = 256, 0.0, 0, 0
    while t_q < 0.1 * seconds:
        t0 = time.perf_counter()
        r = oracle.is_estimate(oq, qbits, 3.0, 1.5, frames, seed=3, frame_base=nq, threads=threads)
        t_q += time.perf_counter() - t0
        eu_q += r["edge_updates"]
        nq += frames
        frames *= 2
    qc_is = {"frames": nq, "seconds": t_q, "edge_updates_per_s": eu_q / t_q}
    single = search_leg(dict(decoder=oracle.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024),
                        2, 0.2 * seconds, 1)
    t_step = sum(mix[k] / legs[k]["edge_updates_per_s"] for k in legs)
    used = sum(l["seconds"] for l in legs.values()) + single["seconds"]
    return {"value": step_eu / t_step, "unit": "edge-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{legs['oms']['patterns']} OMS + {legs['spa']['patterns']} SPA patterns of the "
                      f"same list (fixed shuffle) and {legs['is']['frames']} IS frames, {used:.1f} s; "
                      "value = the GPU step's computed edge-updates over the oracle's time for the "
                      "step (each leg's full-iteration edge-updates at the oracle's rate on that leg)",
            "step_seconds": t_step,
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "legs": legs, "single_thread_spa": single, "qc2640_is": qc_is}


if __name__ == "__main__":
    main()
