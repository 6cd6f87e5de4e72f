"""The streamed-frame decoder (check messages in global memory, APP values in LDS)
against the register-resident decoder and against the oracle.

Both layouts compute the same integers (int8 offset min-sum; Q20 fixed-point
sum-product with exact integer APP sums), so on codes where both fit every
per-pattern output, every TS and every IS frame must be identical.  Codes too
large for the register layout (46x68-base QC codes with column weights 3..5 and
N up to 25.7k; 4x24-base codes with M > 512) are checked against the oracle:
bit-exact for min-sum, k* within 1e-3 relative for sum-product, frame-by-frame
agreement for IS.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")
SPA = dict(max_iter=50, k_max=32 * 1024, k_den=1024)


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2208_05795_amd as tsg
    c = tsg.Context(0)
    yield c
    c.close()


def _ts(recs):
    return [(r.a, r.b, r.orbit, r.first_pattern, r.k_crit, tuple(r.bits)) for r in recs]


def _sample(allp, k, seed):
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(len(allp), min(k, len(allp)), replace=False))
    return np.ascontiguousarray(allp[sel])


def _all_layouts(g, pats, **kw):
    """Register layout, then the streamed layout's gathering and accumulating
    variants (forced)."""
    import paper_2208_05795_amd as tsg
    out = []
    for lay, want, var in ((tsg.LAYOUT_REGISTER, tsg.LAYOUT_REGISTER, None),
                           (tsg.LAYOUT_STREAMED_GATHER, tsg.LAYOUT_STREAMED, 0),
                           (tsg.LAYOUT_STREAMED_ACCUM, tsg.LAYOUT_STREAMED, 1)):
        g.reset_ts()
        r = g.impulse_search(pats, layout=lay, **kw)
        assert r["stats"]["layout"] == want
        if var is not None:
            assert r["stats"]["checks_per_thread"] == var
        out.append(({k: np.asarray(r[k]) for k in KEYS}, _ts(g.collect()), r["stats"]))
    return out


def _same(a, b, label):
    for k in KEYS:
        if not np.array_equal(a[k], b[k]):
            bad = np.nonzero(a[k] != b[k])[0]
            raise AssertionError(f"{label} {k} differs at {bad[:8]}: {a[k][bad[:8]]} vs {b[k][bad[:8]]}")


@pytest.mark.parametrize("name", ["tiny", "peg1008", "qc2640"])
def test_layouts_identical_oms(ctx, oracle_mod, name):
    code = {"tiny": workloads.tiny_code, "peg1008": workloads.peg1008_code,
            "qc2640": workloads.qc2640_code}[name]()
    oc = oracle_mod.OCode(code)
    allp = oracle_mod.pattern_list(oc, [1, 2] if name == "tiny" else [1, 2, 3])
    pats = allp if name == "tiny" else _sample(allp, 3000, 21)
    _say(f"{name} OMS register vs streamed, {len(pats)} patterns")
    g = ctx.load_code(code)
    (ra, ta, sa), (rb, tb, sb), (rc, tc, sc) = _all_layouts(g, pats, a_max=12)
    for r, t, st, lab in ((rb, tb, sb, "gather"), (rc, tc, sc, "accum")):
        _same(ra, r, f"{name} {lab}")
        assert ta == t
        # both layouts' fixed-point exits stop at the first iteration whose
        # messages equal the last one's: the same iterations are computed
        assert sa["decodes"] == st["decodes"]
        assert sa["edge_updates"] == st["edge_updates"], (lab, sa["edge_updates"], st["edge_updates"])
    _say(f"  identical: {len(ta)} TS, {sa['edge_updates']:.3e} edge-updates; decode ms register "
         f"{sa['decode_ms']:.2f} streamed gather {sb['decode_ms']:.2f} accum {sc['decode_ms']:.2f}")
    g.free()


@pytest.mark.parametrize("name", ["peg1008", "qc2640"])
def test_layouts_identical_spa(ctx, oracle_mod, name):
    import paper_2208_05795_amd as tsg
    code = {"peg1008": workloads.peg1008_code, "qc2640": workloads.qc2640_code}[name]()
    oc = oracle_mod.OCode(code)
    pats = _sample(oracle_mod.pattern_list(oc, [1, 2, 3]), 400, 22)
    _say(f"{name} SPA register vs streamed, {len(pats)} patterns")
    g = ctx.load_code(code)
    (ra, ta, sa), (rb, tb, sb), (rc, tc, sc) = _all_layouts(g, pats, decoder=tsg.DEC_SPA, a_max=12, **SPA)
    for r, t, st, lab in ((rb, tb, sb, "gather"), (rc, tc, sc, "accum")):
        _same(ra, r, f"{name} {lab}")
        assert ta == t
        assert sa["edge_updates"] == st["edge_updates"], (lab, sa["edge_updates"], st["edge_updates"])
    _say(f"  identical: {len(ta)} TS, {sa['edge_updates']:.3e} edge-updates; decode ms register {sa['decode_ms']:.2f} "
         f"streamed gather {sb['decode_ms']:.2f} accum {sc['decode_ms']:.2f}")
    g.free()


@pytest.mark.parametrize("name", ["peg1008", "qc2640"])
def test_layouts_identical_is(ctx, oracle_mod, name):
    import paper_2208_05795_amd as tsg
    code = {"peg1008": workloads.peg1008_code, "qc2640": workloads.qc2640_code}[name]()
    g = ctx.load_code(code)
    bits = [int(x) for x in g.csr()[1][:4]]   # the variables of check 0 (a 4-subset)
    res = [g.is_estimate(bits, 1.0, 2.0, 3000, seed=5, stream=2, want_fail=True, layout=lay)
           for lay in (tsg.LAYOUT_REGISTER, tsg.LAYOUT_STREAMED_GATHER, tsg.LAYOUT_STREAMED_ACCUM)]
    assert res[0]["stats"]["layout"] == tsg.LAYOUT_REGISTER
    for var, r in ((0, res[1]), (1, res[2])):
        assert r["stats"]["layout"] == tsg.LAYOUT_STREAMED and r["stats"]["checks_per_thread"] == var
        assert np.array_equal(res[0]["fail"], r["fail"])
        for f in ("p_hat", "var", "sum_w", "sum_w2", "n_fail"):
            assert res[0][f] == r[f], f
        # the same fixed-point iterations in both layouts
        assert res[0]["stats"]["edge_updates"] == r["stats"]["edge_updates"]
    _say(f"{name} IS register vs streamed identical: p {res[0]['p_hat']:.4e}, "
         f"{int(res[0]['n_fail'])} failures")
    assert res[0]["n_fail"] > 0
    g.free()


def test_qc_index_path(ctx):
    """The streamed decoder of a QC code computes its indices from the
    circulant tables (switched on by the loader only after every computed index
    matched the index tables); a CSR code keeps the tables."""
    pool = sorted(workloads.serving_pool(), key=lambda c: c.n)
    wide = [c for c in workloads.batch_codes() if c.mb == 4 and c.nb == 24][0]
    for code, want in ((workloads.peg1008_code(), 0), (workloads.tiny_code(), 1),
                       (workloads.qc2640_code(), 1), (pool[0], 1), (pool[-1], 1), (wide, 1)):
        g = ctx.load_code(code)
        assert g.info["streamed_qc"] == want, code.name
        g.free()


@pytest.fixture(scope="module")
def pool():
    return {c.name: c for c in workloads.serving_pool()}


def _largest(pool):
    return max(pool.values(), key=lambda c: c.n)


def _smallest(pool):
    return min(pool.values(), key=lambda c: c.n)


@pytest.mark.parametrize("which", ["smallest", "largest"])
def test_serving_code_oms_vs_oracle(ctx, oracle_mod, pool, which):
    import paper_2208_05795_amd as tsg
    code = (_smallest if which == "smallest" else _largest)(pool)
    oc = oracle_mod.OCode(code)
    singles = _sample(oracle_mod.patterns(oc, 1).reshape(-1, 1), 8, 30)
    singles = np.hstack([singles, np.full_like(singles, -1)])
    pats = np.ascontiguousarray(np.concatenate([singles, _sample(oracle_mod.patterns(oc, 2), 24, 31)])
                                .astype(np.int32))
    g = ctx.load_code(code)
    # 20 iterations (impulses on these codes are corrected), then 2 iterations
    # from which most impulses fail, so bisection and extraction run as well
    # the smallest code also through both streamed variants (the largest only
    # fits the gathering one)
    layouts = [tsg.LAYOUT_AUTO] + ([tsg.LAYOUT_STREAMED_GATHER, tsg.LAYOUT_STREAMED_ACCUM]
                                   if which == "smallest" else [])
    for kw in (dict(max_iter=20), dict(max_iter=2, collect_from_iter=1)):
        _say(f"{code.name} (n={code.n}, m={code.m}) OMS vs oracle, {len(pats)} patterns, {kw}")
        ref = oracle_mod.search(oc, pats, a_max=12, **kw)
        for lay in layouts:
            g.reset_ts()
            got = g.impulse_search(pats, a_max=12, layout=lay, **kw)
            if code.n > 20000:
                assert got["stats"]["layout"] == tsg.LAYOUT_STREAMED
            for k in KEYS:
                assert np.array_equal(np.asarray(got[k]), ref[k]), (lay, k)
            assert _ts(g.collect()) == _ts(ref["ts"])
            assert got["stats"]["edge_updates"] <= ref["edge_updates"]   # fixed-point exit
        _say(f"  bit-exact ({len(layouts)} layouts); {len(ref['ts'])} TS, "
             f"failing patterns {(ref['k_crit'] >= 0).sum()}")
    g.free()


def test_serving_code_spa_vs_oracle(ctx, oracle_mod, pool):
    import paper_2208_05795_amd as tsg
    code = sorted(pool.values(), key=lambda c: c.n)[1]
    oc = oracle_mod.OCode(code)
    pats = _sample(oracle_mod.patterns(oc, 2), 12, 32)
    _say(f"{code.name} (n={code.n}) SPA streamed vs oracle, {len(pats)} patterns")
    ref = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, a_max=12, **SPA)
    g = ctx.load_code(code)
    got = g.impulse_search(pats, decoder=tsg.DEC_SPA, a_max=12, layout=tsg.LAYOUT_STREAMED, **SPA)
    kg, ko = np.asarray(got["k_crit"]), ref["k_crit"]
    rel = np.abs(kg - ko) / np.maximum(ko, 1)
    ok = ((kg == -1) & (ko == -1)) | ((kg >= 0) & (ko >= 0) & (rel <= 1e-3))
    _say(f"  {ok.sum()}/{len(ok)} within 1e-3, exact {(kg == ko).sum()}")
    assert ok.all()
    for r in g.collect():
        assert oracle_mod.count_b(oc, r.bits) == r.b
        assert tuple(oracle_mod.tree(oc, r.bits)) == r.bits
    g.free()


def test_serving_code_is_vs_oracle(ctx, oracle_mod, pool):
    import paper_2208_05795_amd as tsg
    code = _smallest(pool)
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    rp, col = g.csr()
    bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
    K = 3000
    ref = oracle_mod.is_estimate(oc, bits, 2.5, 1.0, K, seed=13, stream=1, want_fail=True)
    got = g.is_estimate(bits, 2.5, 1.0, K, seed=13, stream=1, want_fail=True,
                        layout=tsg.LAYOUT_STREAMED)
    agree = (got["fail"] == ref["fail"]).mean()
    _say(f"{code.name} IS streamed: p gpu {got['p_hat']:.4e} oracle {ref['p_hat']:.4e} "
         f"agreement {agree:.5f}")
    assert agree >= 0.995
    inside = ref["ci_lo"] <= got["p_hat"] <= ref["ci_hi"]
    close = abs(got["p_hat"] - ref["p_hat"]) <= 0.02 * abs(ref["p_hat"]) + 1e-300
    assert inside or close
    g.free()


def test_wide_check_code_vs_oracle(ctx, oracle_mod):
    """A 4x24-base code with more checks than a register workgroup holds."""
    import paper_2208_05795_amd as tsg
    codes = [c for c in workloads.batch_codes() if c.mb == 4 and c.nb == 24]
    code = max(codes, key=lambda c: c.m)
    oc = oracle_mod.OCode(code)
    pats = _sample(oracle_mod.patterns(oc, 2), 24, 33)
    _say(f"{code.name} (n={code.n}, m={code.m}, dc=24) OMS vs oracle")
    ref = oracle_mod.search(oc, pats, a_max=12)
    g = ctx.load_code(code)
    got = g.impulse_search(pats, a_max=12)
    assert got["stats"]["layout"] == tsg.LAYOUT_STREAMED
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k]), ref[k]), k
    assert _ts(g.collect()) == _ts(ref["ts"])
    g.free()


def test_forced_layout_that_does_not_fit(ctx, pool):
    import paper_2208_05795_amd as tsg
    g = ctx.load_code(_largest(pool))
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.array([[0]], dtype=np.int32), layout=tsg.LAYOUT_REGISTER)
    with pytest.raises(tsg.TsgError):   # two LDS arrays of 25.7k sums do not fit
        g.impulse_search(np.array([[0]], dtype=np.int32), layout=tsg.LAYOUT_STREAMED_ACCUM)
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.array([[0]], dtype=np.int32), layout=7)
    g.free()
