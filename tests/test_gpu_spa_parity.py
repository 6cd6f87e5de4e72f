"""Element-by-element parity of the sum-product impulse search (Section III:
bisection on the impulse amplitude, extraction of S1 = Tree(S u I) and
S2 = Tree(TS(S u I))) against the double-precision oracle.

The bar on the critical amplitude is eps* = k*/1024 within 1e-3 relative.
Beyond it, on the PEG-1008 code, the QC-2640 triples and a 46x68-base serving
code (streamed layout), every per-pattern output (k*, iterations at k* and at
the last success, first minimum-syndrome iteration, candidate count) and the
ordered TS list (a, b, orbit, first pattern, smallest k*, bits) must be
identical.  Only patterns whose oracle outputs themselves change when the
oracle's messages are rounded to the device's 2^-20 grid (the conditioning
probe of or_decode_spa_grid) may be excluded from that, counted and reported
(observed: none); the TS lists are then compared on a rerun of both sides over
the remaining patterns.

On the tiny QC code (N = 96), the sum-product decodes at large impulse
amplitudes are chaotic, and the outputs other than k* are held to a
statistical bar set by the oracle's own sensitivity (_tiny_statistical).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")
SPA = dict(max_iter=50, k_max=32 * 1024, k_den=1024)
# the device stores sum-product messages and APP values on the 2^-20 grid
GRID = 20


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


def _compare(g, oracle_mod, oc, pats, a_max, label, layout=0, max_excluded=0.0, **kw):
    """Runs both sides on pats; returns (number compared, number excluded).

    A pattern is compared element by element when its oracle outputs do not
    depend on the message precision: the double-precision search and its
    conditioning probe (messages rounded to the device's 2^-20 grid) agree on
    it.  The others are excluded, counted, and held to the eps* tolerance only."""
    import paper_2208_05795_amd as tsg
    pats = np.ascontiguousarray(pats, dtype=np.int32)
    kw = dict(SPA, **kw)
    ref = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, a_max=a_max, **kw)
    probe = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, a_max=a_max,
                              spa_grid=GRID, **kw)
    cond = np.ones(len(pats), dtype=bool)
    for k in KEYS:
        cond &= ref[k] == probe[k]
    g.reset_ts()
    got = g.impulse_search(pats, decoder=tsg.DEC_SPA, a_max=a_max, layout=layout, **kw)
    got = {k: np.asarray(got[k]) for k in KEYS}
    kg, ko = got["k_crit"], ref["k_crit"]
    rel = np.abs(kg - ko) / np.maximum(ko, 1)
    within = ((kg == -1) & (ko == -1)) | ((kg >= 0) & (ko >= 0) & (rel <= 1e-3))
    assert within.all(), (label, np.nonzero(~within)[0][:10])
    n_ex = int((~cond).sum())
    diff = {k: int((got[k] != ref[k]).sum()) for k in KEYS}
    diff_cond = {k: int((got[k][cond] != ref[k][cond]).sum()) for k in KEYS}
    _say(f"{label}: {len(pats)} patterns, {int((ko >= 0).sum())} failing; k* exact on "
         f"{int((kg == ko).sum())}; precision-sensitive (excluded) {n_ex}; "
         f"differences on all patterns {diff}, on the compared ones {diff_cond}")
    assert n_ex <= max_excluded * len(pats), (label, n_ex)
    for k in KEYS:
        bad = np.nonzero(got[k][cond] != ref[k][cond])[0]
        idx = np.nonzero(cond)[0][bad[:10]]
        assert len(bad) == 0, (label, k, idx, got[k][idx], ref[k][idx])
    if n_ex == 0:
        gts, rts = _ts(g.collect()), _ts(ref["ts"])
    else:
        sub = np.ascontiguousarray(pats[cond])
        ref2 = oracle_mod.search(oc, sub, decoder=oracle_mod.DEC_SPA, a_max=a_max, **kw)
        g.reset_ts()
        g.impulse_search(sub, decoder=tsg.DEC_SPA, a_max=a_max, layout=layout, **kw)
        gts, rts = _ts(g.collect()), _ts(ref2["ts"])
    if gts != rts:
        gs, rs = set(gts), set(rts)
        _say(f"  TS lists differ: {len(gs - rs)} only on the device, {len(rs - gs)} only in "
             f"the oracle: {sorted(gs - rs)[:3]} / {sorted(rs - gs)[:3]}")
    assert gts == rts, (label, len(gts), len(rts))
    _say(f"  per-pattern outputs and {len(rts)} TS identical on {int(cond.sum())} patterns")
    return int(cond.sum()), n_ex


def _tiny_statistical(g, oracle_mod, oc, pats, label, **kw):
    """The tiny code's sum-product decodes at impulse amplitudes up to 32 often
    oscillate for all 50 iterations, and there the per-pattern outputs other
    than k* depend on the arithmetic's precision: the double-precision oracle
    changes them on a fifth of the patterns when its messages are rounded to
    the 2^-19 grid.  Bar: k* within 1e-3 on every pattern (observed: exact),
    and the device disagrees with the oracle on no more patterns, and on no
    more TS, than the oracle disagrees with itself under the 2^-19..2^-21
    message grids."""
    import paper_2208_05795_amd as tsg
    pats = np.ascontiguousarray(pats, dtype=np.int32)
    kw = dict(SPA, **kw)
    ref = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, a_max=6, **kw)
    g.reset_ts()
    got = g.impulse_search(pats, decoder=tsg.DEC_SPA, a_max=6, **kw)
    got = {k: np.asarray(got[k]) for k in KEYS}
    assert np.array_equal(got["k_crit"], ref["k_crit"]), label

    def n_diff(x):
        d = np.zeros(len(pats), dtype=bool)
        for k in KEYS:
            d |= np.asarray(x[k]) != ref[k]
        return int(d.sum())

    def ts_diff(lst):
        a, b = set(_ts(lst)), set(_ts(ref["ts"]))
        return len(a ^ b)

    dev_p, dev_t = n_diff(got), ts_diff(g.collect())
    probes = []
    for grid in (19, 20, 21):
        pr = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, a_max=6, spa_grid=grid, **kw)
        probes.append((grid, n_diff(pr), ts_diff(pr["ts"])))
    _say(f"{label}: {len(pats)} patterns, {len(ref['ts'])} TS; device vs oracle: {dev_p} "
         f"patterns, {dev_t} TS differ; oracle vs its message-grid probes (grid, patterns, TS): "
         f"{probes}")
    assert dev_p <= max(p for _, p, _ in probes)
    assert dev_t <= max(t for _, _, t in probes)


def test_spa_parity_tiny_all(ctx, oracle_mod, tiny):
    code, oc = tiny
    pats = oracle_mod.pattern_list(oc, [1, 2])[::2]
    g = ctx.load_code(code)
    _tiny_statistical(g, oracle_mod, oc, pats, "tiny SPA, every other single and pair")
    g.free()


def test_spa_parity_tiny_critical_mode(ctx, oracle_mod, tiny):
    code, oc = tiny
    pats = oracle_mod.pattern_list(oc, [1, 2])[1::3]
    g = ctx.load_code(code)
    _tiny_statistical(g, oracle_mod, oc, pats, "tiny SPA, critical extraction",
                      extract_mode=oracle_mod.EXTRACT_CRITICAL)
    g.free()


def test_spa_parity_peg1008(ctx, oracle_mod):
    """At least 150 patterns, at least 60 of them failing at some amplitude."""
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    allp = g.pattern_list([1, 2, 3])
    rng = np.random.default_rng(41)
    probe = np.sort(rng.choice(len(allp), 4096, replace=False))
    r = g.impulse_search(np.ascontiguousarray(allp[probe]), decoder=tsg.DEC_SPA, a_max=12, **SPA)
    failing = probe[np.asarray(r["k_crit"]) >= 0]
    pick = np.unique(np.concatenate([rng.choice(probe, 200, replace=False),
                                     rng.choice(failing, min(200, len(failing)), replace=False)]))
    pats = np.ascontiguousarray(allp[pick])
    n_cmp, _ = _compare(g, oracle_mod, oc, pats, 12, "PEG-1008 SPA", max_excluded=0.02)
    assert len(pats) >= 150 and n_cmp >= 300
    g.free()


def test_spa_parity_qc2640_triples(ctx, oracle_mod):
    code = workloads.qc2640_code()
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    allp = g.make_patterns(3)
    rng = np.random.default_rng(42)
    pats = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 160, replace=False))])
    _compare(g, oracle_mod, oc, pats, 12, "QC-2640 SPA triples", max_excluded=0.02)
    g.free()


def test_spa_parity_serving_code(ctx, oracle_mod):
    """A 46x68-base code with column weights 3..5 in the streamed layout."""
    import paper_2208_05795_amd as tsg
    pool = workloads.serving_pool()
    code = sorted(pool, key=lambda c: c.n)[1]
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    allp = oracle_mod.pattern_list(oc, [1, 2])
    rng = np.random.default_rng(43)
    pats = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 40, replace=False))])
    _compare(g, oracle_mod, oc, pats, 12, f"{code.name} (n={code.n}) SPA streamed",
             layout=tsg.LAYOUT_STREAMED, max_excluded=0.05)
    g.free()
