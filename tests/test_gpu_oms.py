"""GPU parity of the int8 offset-min-sum impulse search against the CPU oracle.

The bar is bit-exact: critical amplitudes, iteration counts, first minimum-
syndrome iterations, candidate counts and the whole ordered TS list.
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


def _ts(recs):
    return [(r.a, r.b, r.orbit, r.first_pattern, r.k_crit, tuple(r.bits)) for r in recs]


def _same(got, ref):
    for k in KEYS:
        if not np.array_equal(np.asarray(got[k]), np.asarray(ref[k])):
            bad = np.nonzero(np.asarray(got[k]) != np.asarray(ref[k]))[0]
            raise AssertionError(f"{k} differs at {bad[:10]}: gpu {np.asarray(got[k])[bad[:10]]} "
                                 f"oracle {np.asarray(ref[k])[bad[:10]]}")


@pytest.mark.parametrize("name", ["tiny", "tiny_z8", "peg1008", "qc2640", "table5"])
def test_code_load_matches_oracle(ctx, oracle_mod, name):
    code = {"tiny": workloads.tiny_code, "tiny_z8": workloads.tiny_code_z8,
            "peg1008": workloads.peg1008_code, "qc2640": workloads.qc2640_code,
            "table5": workloads.table5_code1}[name]()
    _say(f"load {name}")
    g = ctx.load_code(code)
    oc = oracle_mod.OCode(code)
    rp, col = g.csr()
    orp, ocol = oc.csr()
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    assert (g.n, g.m, g.e, g.girth) == (oc.n, oc.m, oc.e, oc.girth)
    g.free()


def test_tiny_triples_large_table(ctx, oracle_mod, tiny):
    """Singles, pairs and tree-path triples of the tiny code with a_max 12:
    about 14,000 TS, so the ordered read-out takes the multi-launch sort of
    large tables (tables of up to 8192 sets sort in one launch, as every
    other test here does)."""
    code, oc = tiny
    pats = oracle_mod.pattern_list(oc, [1, 2, 3])
    ref = oracle_mod.search(oc, pats, a_max=12)
    _say(f"tiny triples, {len(pats)} patterns, {len(ref['ts'])} TS")
    assert len(ref["ts"]) > 8192
    g = ctx.load_code(code)
    got = g.impulse_search(pats, a_max=12)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    g.free()


def test_patterns_match_oracle(ctx, oracle_mod):
    for code in (workloads.tiny_code(), workloads.peg1008_code()):
        g = ctx.load_code(code)
        oc = oracle_mod.OCode(code)
        for kind in (1, 2, 3):
            assert np.array_equal(g.make_patterns(kind), oracle_mod.patterns(oc, kind)), kind
        g.free()


def test_tiny_full_search_bit_exact(ctx, oracle_mod, tiny, tiny_search):
    """Tiny QC code: every single and every pair within distance 4, OMS int8,
    offset 1, 20 iterations, 3 dB, grid k/16 up to 32, a_max 6."""
    code, oc = tiny
    pats, ref = tiny_search
    _say(f"tiny full search, {len(pats)} patterns")
    g = ctx.load_code(code)
    got = g.impulse_search(pats, a_max=6)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    # the oracle computes every iteration; the fixed-point exit may compute fewer
    assert got["stats"]["edge_updates"] <= ref["edge_updates"]
    assert got["stats"]["decodes"] == ref["decodes"]
    full = g.impulse_search(pats, a_max=6, full_iterations=True)
    assert full["stats"]["edge_updates"] == ref["edge_updates"]
    g.free()


@pytest.fixture(scope="module")
def peg_sample(oracle_mod):
    code = workloads.peg1008_code()
    oc = oracle_mod.OCode(code)
    allp = oracle_mod.pattern_list(oc, [1, 2, 3])
    rng = np.random.default_rng(21)
    idx = np.sort(rng.choice(len(allp), 1500, replace=False))
    pats = np.ascontiguousarray(allp[idx])
    ref = oracle_mod.search(oc, pats, a_max=12)
    return code, oc, pats, ref


def test_peg_sample_bit_exact(ctx, peg_sample):
    code, oc, pats, ref = peg_sample
    _say(f"peg1008 sample, {len(pats)} patterns")
    g = ctx.load_code(code)
    got = g.impulse_search(pats, a_max=12)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    g.free()


def test_critical_mode_bit_exact(ctx, oracle_mod, tiny, tiny_search):
    code, oc = tiny
    pats, _ = tiny_search
    ref = oracle_mod.search(oc, pats, a_max=6, extract_mode=oracle_mod.EXTRACT_CRITICAL)
    _say("tiny critical-mode search")
    g = ctx.load_code(code)
    import paper_2208_05795_amd as tsg
    got = g.impulse_search(pats, a_max=6, extract_mode=tsg.EXTRACT_CRITICAL)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    g.free()


@pytest.mark.parametrize("opts", [dict(max_iter=1), dict(max_iter=3, a_max=1),
                                  dict(collect_from_iter=1, a_max=4), dict(oms_offset=0),
                                  dict(oms_offset=3, k_max=200), dict(ebn0_db=5.0, a_max=5),
                                  dict(max_iter=64, a_max=16)])
def test_option_edges_bit_exact(ctx, oracle_mod, tiny, tiny_search, opts):
    code, oc = tiny
    pats, _ = tiny_search
    pats = pats[::7]
    ref = oracle_mod.search(oc, pats, **opts)
    _say(f"tiny search {opts}")
    g = ctx.load_code(code)
    got = g.impulse_search(pats, **opts)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    g.free()


def test_wide_and_padded_patterns(ctx, oracle_mod, tiny):
    code, oc = tiny
    rng = np.random.default_rng(4)
    pats = np.full((64, 16), -1, dtype=np.int32)
    for i in range(64):
        w = int(rng.integers(0, 17))
        pats[i, :w] = rng.choice(oc.n, w, replace=False)
    ref = oracle_mod.search(oc, pats, a_max=8)
    _say("tiny width-16 patterns")
    g = ctx.load_code(code)
    got = g.impulse_search(pats, a_max=8)
    _same(got, ref)
    assert _ts(g.collect()) == _ts(ref["ts"])
    # a row of -1 is no impulse at all: decoded at once at every amplitude
    empty = np.nonzero((pats < 0).all(axis=1))[0]
    assert (np.asarray(got["k_crit"])[empty] == -1).all()
    g.free()


def test_empty_and_invalid_inputs(ctx, tiny):
    import paper_2208_05795_amd as tsg
    code, oc = tiny
    g = ctx.load_code(code)
    got = g.impulse_search(np.zeros((0, 2), dtype=np.int32))
    assert all(len(got[k]) == 0 for k in KEYS)
    for bad in (np.array([[96]]), np.array([[-2]])):
        with pytest.raises(tsg.TsgError):
            g.impulse_search(bad)
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.zeros((1, 17), dtype=np.int32))
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.zeros((1, 1), dtype=np.int32), k_den=8)
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.zeros((1, 1), dtype=np.int32), a_max=17)
    for bad in (dict(ebn0_db=float("nan")), dict(llr_scale=float("inf"))):
        with pytest.raises(tsg.TsgError):
            g.impulse_search(np.zeros((1, 1), dtype=np.int32), **bad)
    assert g.collect() == []
    g.free()


def test_device_memory_path_and_determinism(ctx, oracle_mod, peg_sample):
    import torch
    code, oc, pats, ref = peg_sample
    _say("peg1008 sample from device memory, twice")
    g = ctx.load_code(code)
    dp = torch.from_numpy(pats).cuda()
    a = g.impulse_search(dp, a_max=12)
    t1 = _ts(g.collect())
    g.reset_ts()
    b = g.impulse_search(dp, a_max=12)
    t2 = _ts(g.collect())
    for k in KEYS:
        assert torch.equal(a[k], b[k])
        assert np.array_equal(a[k].cpu().numpy(), ref[k])
    assert t1 == t2 == _ts(ref["ts"])
    g.free()


def test_qc_shift_invariance(ctx, tiny, tiny_search):
    code, oc = tiny
    pats, ref = tiny_search
    z = code.z
    sp = np.where(pats >= 0, (pats // z) * z + (pats % z + 5) % z, -1).astype(np.int32)
    _say("tiny shifted patterns")
    g = ctx.load_code(code)
    got = g.impulse_search(sp, a_max=6)
    for k in KEYS:
        assert np.array_equal(got[k], ref[k]), k
    assert [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in g.collect()] == \
        [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in ref["ts"]]
    g.free()


def test_table_accumulates_across_calls(ctx, oracle_mod, tiny, tiny_search):
    """Two searches on halves merge into the same table as one search on all."""
    code, oc = tiny
    pats, ref = tiny_search
    h = len(pats) // 2
    g = ctx.load_code(code)
    g.impulse_search(pats[:h], a_max=6)
    r2 = g.impulse_search(pats[h:], a_max=6)
    got = g.collect()
    # first_pattern is relative to each call; compare the rest
    assert [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in got] == \
        [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in ref["ts"]]
    assert np.array_equal(r2["k_crit"], ref["k_crit"][h:])
    g.free()
