"""The fixed-point exit of the decoders: a decode whose check messages do not
change in an iteration stops computing and fills in its remaining iterations
(each repeats the last).  Register layout: a hash of each thread's messages
triggers a verifying iteration; streamed layout: every check compares the old
message it reads with the new one it writes.  Every output must equal that of
the same call with every iteration computed (full_iterations), bit for bit:
per-pattern arrays, the TS table, IS estimates and failure flags; the exit
must also actually fire (fewer computed edge-updates) where decodes fail.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2208_05795_amd as tsg
    c = tsg.Context(0)
    yield c
    c.close()


def _search_both(ctx, code, pats, **kw):
    out = []
    for full in (True, False):
        g = ctx.load_code(code)
        r = g.impulse_search(pats, full_iterations=full, **kw)
        recs, bits = g.collect_arrays()
        out.append((r, recs, bits))
        g.free()
    return out


def _assert_same(full, fast, label):
    (r0, recs0, bits0), (r1, recs1, bits1) = full, fast
    for k in KEYS:
        assert np.array_equal(np.asarray(r0[k]), np.asarray(r1[k])), (label, k)
    assert np.array_equal(recs0, recs1), label
    assert np.array_equal(bits0, bits1), label
    e0, e1 = r0["stats"]["edge_updates"], r1["stats"]["edge_updates"]
    _say(f"{label}: identical; computed edge-updates {e0} full, {e1} with the exit "
         f"({e1 / max(e0, 1):.3f})")
    return e0, e1


def test_spa_peg_exit_identical(ctx):
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    g = ctx.load_code(code)
    allp = g.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS, tsg.PAT_TRIPLES])
    g.free()
    rng = np.random.default_rng(21)
    pats = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 4096, replace=False))])
    kw = dict(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12,
              layout=tsg.LAYOUT_REGISTER)
    e0, e1 = _assert_same(*_search_both(ctx, code, pats, **kw), "peg SPA")
    assert e1 < e0   # failing SPA decodes reach fixed points


def test_spa_qc2640_exit_identical(ctx):
    import paper_2208_05795_amd as tsg
    code = workloads.qc2640_code()
    g = ctx.load_code(code)
    pats = g.make_patterns(tsg.PAT_TRIPLES | tsg.PAT_QC_ORBITS)
    g.free()
    kw = dict(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12,
              layout=tsg.LAYOUT_REGISTER)
    _assert_same(*_search_both(ctx, code, pats, **kw), "qc2640 SPA orbit representatives")


@pytest.mark.parametrize("scale", [4.0, 1.2])
def test_oms_exit_identical(ctx, scale):
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    g = ctx.load_code(code)
    pats = g.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS])
    g.free()
    kw = dict(decoder=tsg.DEC_OMS, max_iter=20, llr_scale=scale, a_max=12,
              layout=tsg.LAYOUT_REGISTER)
    _assert_same(*_search_both(ctx, code, pats, **kw), f"peg OMS scale {scale}")


@pytest.mark.parametrize("which", ["peg", "qc2640"])
def test_lnms_exit_identical(ctx, which):
    """The layered decoder's exit (a sweep that leaves every message and APP
    value unchanged), at a weak channel scale where every impulse fails."""
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code() if which == "peg" else workloads.qc2640_code()
    g = ctx.load_code(code)
    if which == "peg":
        pats = g.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS])
    else:
        pats = g.make_patterns(tsg.PAT_TRIPLES)[::8]
    g.free()
    kw = dict(decoder=tsg.DEC_LNMS, max_iter=20, llr_scale=0.3, k_max=512, k_den=16, a_max=12)
    e0, e1 = _assert_same(*_search_both(ctx, code, pats, **kw), f"{which} layered min-sum x0.3")
    assert e1 <= e0


def test_is_exit_identical(ctx):
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    g = ctx.load_code(code)
    g.impulse_search(g.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS])[:2048], decoder=tsg.DEC_SPA,
                     max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12)
    ts = g.collect()
    assert ts
    bits = list(ts[0].bits)
    res = []
    for full in (True, False):
        r = g.is_estimate(bits, 3.0, -1.0, 8192, seed=5, want_fail=True,
                          layout=tsg.LAYOUT_REGISTER, full_iterations=full)
        res.append(r)
    g.free()
    a, b = res
    assert np.array_equal(a["fail"], b["fail"])
    for k in ("p_hat", "var", "sum_w", "sum_w2", "n_fail", "shift_used"):
        assert a[k] == b[k], k
    _say(f"IS: identical; computed edge-updates {a['stats']['edge_updates']} full, "
         f"{b['stats']['edge_updates']} with the exit")


def test_batch_exit_identical(ctx):
    """Batched search and IS jobs (shared persistent launches, one scratch arena
    per shape group) give the same outputs with and without the exit."""
    import paper_2208_05795_amd as tsg
    peg = ctx.load_code(workloads.peg1008_code())
    qc = ctx.load_code(workloads.qc2640_code())
    rng = np.random.default_rng(4)
    allp = peg.pattern_list([tsg.PAT_PAIRS, tsg.PAT_TRIPLES])
    pp = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 2048, replace=False))])
    qp = qc.make_patterns(tsg.PAT_TRIPLES | tsg.PAT_QC_ORBITS)
    spa = dict(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12)
    peg.impulse_search(pp[:512], **spa)
    bits = list(peg.collect()[0].bits)
    outs = []
    for full in (True, False):
        jobs = [("search", peg, pp, dict(spa, full_iterations=full)),
                ("search", qc, qp, dict(spa, full_iterations=full)),
                ("is", peg, bits, dict(ebn0_db=3.0, shift=-1.0, n_frames=4096, seed=9,
                                       full_iterations=full))]
        ids = ctx.run_batch(jobs)
        res = []
        for j in ids:
            info = ctx.poll(j)
            if info["n_patterns"]:
                o = ctx.job_outputs(j, arrays=True)
                res.append(({k: np.asarray(o[k]) for k in KEYS}, o["ts_recs"], o["ts_bits"]))
            else:
                res.append(info["is"])
            ctx.release(j)
        outs.append(res)
    for a, b in zip(*outs):
        if isinstance(a, dict):
            assert a == b
        else:
            for k in KEYS:
                assert np.array_equal(a[0][k], b[0][k]), k
            assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    _say("batch: identical with and without the exit")
    peg.free()
    qc.free()


@pytest.mark.parametrize("variant", ["gather", "accum"])
def test_streamed_spa_exit_identical(ctx, variant):
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    g = ctx.load_code(code)
    allp = g.pattern_list([tsg.PAT_SINGLES, tsg.PAT_PAIRS, tsg.PAT_TRIPLES])
    g.free()
    rng = np.random.default_rng(23)
    pats = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 1024, replace=False))])
    lay = tsg.LAYOUT_STREAMED_GATHER if variant == "gather" else tsg.LAYOUT_STREAMED_ACCUM
    kw = dict(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12, layout=lay)
    e0, e1 = _assert_same(*_search_both(ctx, code, pats, **kw), f"peg SPA streamed {variant}")
    assert e1 < e0


def test_streamed_oms_exit_identical(ctx):
    import paper_2208_05795_amd as tsg
    code = workloads.qc2640_code()
    g = ctx.load_code(code)
    pats = g.make_patterns(tsg.PAT_TRIPLES)[::16]
    g.free()
    kw = dict(decoder=tsg.DEC_OMS, max_iter=20, llr_scale=1.2, a_max=12,
              layout=tsg.LAYOUT_STREAMED)
    _assert_same(*_search_both(ctx, code, pats, **kw), "qc2640 OMS streamed x1.2")


@pytest.mark.parametrize("variant", ["gather", "accum"])
def test_streamed_is_exit_identical(ctx, variant):
    """IS frames on a 46x68-base serving code (column weights 3..5) that only
    the streamed layout holds at its size, at an SNR where frames fail."""
    import paper_2208_05795_amd as tsg
    pool = workloads.serving_pool()
    code = sorted(pool, key=lambda c: c.n)[1]
    g = ctx.load_code(code)
    rp, col = g.csr()
    bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
    lay = tsg.LAYOUT_STREAMED_GATHER if variant == "gather" else tsg.LAYOUT_STREAMED_ACCUM
    res = []
    for full in (True, False):
        res.append(g.is_estimate(bits, 1.5, 1.0, 4096, seed=5, want_fail=True, layout=lay,
                                 full_iterations=full))
    g.free()
    a, b = res
    assert np.array_equal(a["fail"], b["fail"])
    for k in ("p_hat", "var", "sum_w", "sum_w2", "n_fail", "shift_used"):
        assert a[k] == b[k], k
    e0, e1 = a["stats"]["edge_updates"], b["stats"]["edge_updates"]
    _say(f"IS streamed {variant} ({code.name}): identical, {int(a['n_fail'])} failing frames; "
         f"computed edge-updates {e0} full, {e1} with the exit ({e1 / max(e0, 1):.3f})")
    assert e1 <= e0
