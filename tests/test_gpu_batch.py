"""Batched execution (ts_run_batch): search and IS jobs on codes of uneven size
share persistent launches.  Every job's result must equal the same call run
alone, bit for bit (the kernels compute the same integers; each search job has
its own TS table), including codes that only the streamed decoder holds.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _ts(recs):
    return [(r.a, r.b, r.orbit, r.first_pattern, r.k_crit, tuple(r.bits)) for r in recs]


def _alone(codes, jobs):
    import paper_2208_05795_amd as tsg
    out = []
    with tsg.Context(0) as ctx:
        loaded = {k: ctx.load_code(v) for k, v in codes.items()}
        for kind, name, data, kw in jobs:
            c = loaded[name]
            if kind == "search":
                c.reset_ts()
                r = c.impulse_search(data, **kw)
                out.append(({k: np.asarray(r[k]) for k in KEYS}, _ts(c.collect()),
                            r["stats"]["edge_updates"]))
            else:
                kw = dict(kw)
                r = c.is_estimate(data, kw.pop("ebn0_db"), kw.pop("shift"), kw.pop("n_frames"),
                                  kw.pop("seed"), **kw)
                out.append(r)
    return out


def _batched(codes, jobs, **ctx_kw):
    import paper_2208_05795_amd as tsg
    out = []
    with tsg.Context(0, **ctx_kw) as ctx:
        loaded = {k: ctx.load_code(v) for k, v in codes.items()}
        ids = ctx.run_batch([(kind, loaded[name], data, kw) for kind, name, data, kw in jobs])
        st = ctx.stats()
        for (kind, name, data, kw), jid in zip(jobs, ids):
            info = ctx.poll(jid)
            assert info["state"] == 2 and info["status"] == 0, info
            if kind == "search":
                o = ctx.job_outputs(jid)
                out.append(({k: np.asarray(o[k]) for k in KEYS}, _ts(o["ts"]), info["edge_updates"]))
            else:
                out.append(info["is"])
            ctx.release(jid)
    return out, st


def _compare(jobs, alone, batched):
    for (kind, name, _, kw), a, b in zip(jobs, alone, batched):
        if kind == "search":
            for k in KEYS:
                assert np.array_equal(a[0][k], b[0][k]), (name, kw, k)
            assert a[1] == b[1], (name, kw)
            assert a[2] == b[2], (name, kw, "edge updates")
        else:
            for f in ("p_hat", "var", "sum_w", "sum_w2", "n_fail", "shift_used"):
                assert a[f] == b[f], (name, f)


@pytest.fixture(scope="module")
def mixed(oracle_mod):
    pool = sorted(workloads.serving_pool(), key=lambda c: c.n)
    codes = {"tiny": workloads.tiny_code(), "peg": workloads.peg1008_code(),
             "qc": workloads.qc2640_code(), "s_small": pool[0], "s_big": pool[-1]}
    bc = [c for c in workloads.batch_codes() if c.mb == 4 and c.nb == 24]
    codes["wide"] = min((c for c in bc if c.m > 512), key=lambda c: c.n)
    rng = np.random.default_rng(77)
    jobs = []
    for name, c in codes.items():
        oc = oracle_mod.OCode(c)
        p2 = oracle_mod.patterns(oc, 2)
        sel = np.sort(rng.choice(len(p2), min(len(p2), 600 if c.n < 5000 else 64), replace=False))
        pats = np.ascontiguousarray(p2[sel])
        jobs.append(("search", name, pats, dict(a_max=12)))
        if c.n < 5000:
            jobs.append(("search", name, pats[:96], dict(decoder=1, max_iter=50, k_max=32 * 1024,
                                                          k_den=1024, a_max=12)))
        if name == "s_big":
            jobs.append(("search", name, pats, dict(a_max=12, max_iter=2, collect_from_iter=1)))
        rp, col = oc.csr()
        bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
        jobs.append(("is", name, bits, dict(ebn0_db=2.0, shift=1.5, n_frames=1500, seed=3,
                                            stream=len(jobs))))
    return codes, jobs


def test_batch_equals_alone(mixed):
    codes, jobs = mixed
    _say(f"{len(jobs)} jobs on {len(codes)} codes alone")
    alone = _alone(codes, jobs)
    _say("same jobs in one batch")
    batched, st = _batched(codes, jobs)
    _say(f"  batch: {st['decode_launches']} decode launches for {len(jobs)} jobs, "
         f"{st['edge_updates']:.3e} edge-updates in {st['decode_ms']:.1f} ms")
    _compare(jobs, alone, batched)


def test_batch_of_config4_codes(oracle_mod):
    """Sixteen of the 64 uneven QC codes, each with impulse and IS jobs."""
    codes = {c.name: c for c in workloads.batch_codes()[:16]}
    rng = np.random.default_rng(78)
    jobs = []
    for name, c in codes.items():
        oc = oracle_mod.OCode(c)
        singles = np.stack([np.arange(c.n), np.full(c.n, -1)], axis=1)
        p2 = oracle_mod.patterns(oc, 2)
        sel = np.sort(rng.choice(len(p2), min(len(p2), 256), replace=False))
        pats = np.ascontiguousarray(np.concatenate([singles[:256], p2[sel]]).astype(np.int32))
        jobs.append(("search", name, pats, dict(a_max=12)))
        rp, col = oc.csr()
        bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
        jobs.append(("is", name, bits, dict(ebn0_db=2.0, shift=1.0, n_frames=1024, seed=4,
                                            stream=len(jobs))))
    alone = _alone(codes, jobs)
    batched, st = _batched(codes, jobs)
    _say(f"config-4 sample: {len(jobs)} jobs, {st['decode_launches']} decode launches")
    _compare(jobs, alone, batched)


def test_batch_rejects_bad_job(mixed):
    import paper_2208_05795_amd as tsg
    codes, _ = mixed
    with tsg.Context(0) as ctx:
        c = ctx.load_code(codes["tiny"])
        with pytest.raises(tsg.TsgError):
            ctx.run_batch([("search", c, np.array([[0]], dtype=np.int32), {}),
                           ("search", c, np.array([[96]], dtype=np.int32), {})])
        assert ctx.run_batch([]) == []


def test_batch_eps_shifts_equal_alone():
    """IS jobs whose shift is eps* (the impulse on the whole set): in a batch
    the shifts of all sets of a code come from one search launch; every job
    must equal the same call alone."""
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    with tsg.Context(0) as ctx:
        g = ctx.load_code(code)
        rp, col = g.csr()
        sets = [sorted(int(x) for x in col[rp[r]:rp[r + 1]])[:4] for r in (0, 1, 2)]
        kw = dict(ebn0_db=3.0, shift=-1.0, n_frames=2048, seed=11, max_iter=50)
        alone = [g.is_estimate(b, kw["ebn0_db"], kw["shift"], kw["n_frames"], kw["seed"],
                               max_iter=50, stream=i) for i, b in enumerate(sets)]
        ids = ctx.run_batch([("is", g, b, dict(kw, stream=i)) for i, b in enumerate(sets)])
        for a, jid in zip(alone, ids):
            info = ctx.poll(jid)
            assert info["state"] == 2 and info["status"] == 0, info
            got = info["is"]
            for f in ("shift_used", "p_hat", "var", "sum_w", "sum_w2", "n_fail"):
                assert a[f] == got[f], f
            ctx.release(jid)
        _say(f"eps* shifts {[a['shift_used'] for a in alone]}: batch equals alone")


def test_batch_against_oracle(oracle_mod):
    """Jobs on three small codes in one batch, each compared with the oracle
    directly: OMS searches bit-exact (k*, iteration counts, tmin, candidate
    counts, the ordered TS list), IS estimates within 2% or inside the
    oracle's 95% interval and failure counts within 0.5% of the frames."""
    by_name = {c.name: c for c in workloads.batch_codes()}
    codes = {"tiny": workloads.tiny_code(), "b4x8": by_name["batch35-4x8-z18"],
             "b3x6": by_name["batch54-3x6-z64"]}
    rng = np.random.default_rng(79)
    jobs, refs = [], []
    for name, c in codes.items():
        oc = oracle_mod.OCode(c)
        p2 = oracle_mod.patterns(oc, 2)
        sel = np.sort(rng.choice(len(p2), min(len(p2), 400), replace=False))
        pats = np.ascontiguousarray(p2[sel])
        jobs.append(("search", name, pats, dict(a_max=12)))
        refs.append(oracle_mod.search(oc, pats, a_max=12))
        rp, col = oc.csr()
        bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
        kw = dict(ebn0_db=3.0, shift=1.0, n_frames=3000, seed=5, stream=len(jobs))
        jobs.append(("is", name, bits, kw))
        refs.append(oracle_mod.is_estimate(oc, bits, kw["ebn0_db"], kw["shift"], kw["n_frames"],
                                           seed=kw["seed"], stream=kw["stream"]))
    _say(f"{len(jobs)} jobs on {len(codes)} codes in one batch against the oracle")
    batched, _ = _batched(codes, jobs)
    for (kind, name, _, kw), ref, got in zip(jobs, refs, batched):
        if kind == "search":
            for k in KEYS:
                assert np.array_equal(got[0][k], np.asarray(ref[k])), (name, k)
            assert got[1] == _ts(ref["ts"]), name
        else:
            K = kw["n_frames"]
            _say(f"  IS {name}: p batch {got['p_hat']:.4e} oracle {ref['p_hat']:.4e} "
                 f"ci [{ref['ci_lo']:.3e},{ref['ci_hi']:.3e}] fails {got['n_fail']} / {ref['n_fail']}")
            inside = ref["ci_lo"] <= got["p_hat"] <= ref["ci_hi"]
            close = abs(got["p_hat"] - ref["p_hat"]) <= 0.02 * abs(ref["p_hat"]) + 1e-300
            assert inside or close, name
            assert abs(got["n_fail"] - ref["n_fail"]) <= 0.005 * K, name
