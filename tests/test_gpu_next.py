"""The steps after the IS estimator: automorphism-reduced impulse lists, the TS
spectrum in the form of Tables III/IV, and the union bound on the FER.

* Reduced lists hold exactly one pattern per orbit of the circulant shift (the
  oracle's canonical form of every full-list pattern, computed independently,
  gives the same set), and a search over the reduced list finds the same
  canonical TS, with the same orbit sizes and k*, as over the full list.
* The spectrum equals the counts of the oracle's TS list (bit-exact search).
* The union bound equals sum over sets of orbit x P_hat with the oracle's
  estimates of the same Philox frames, within 2% or the oracle's CI.
* The cycle / EMD spectrum walked on the base matrix reproduces Table II for
  Code 1 and equals the oracle's expanded-graph enumeration on other codes.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2208_05795_amd as tsg
    c = tsg.Context(0)
    yield c
    c.close()


def _ts_key(r):
    """TS identity and the values that do not depend on the pattern list."""
    return (r.a, r.b, r.orbit, r.k_crit, tuple(r.bits))


@pytest.mark.parametrize("name,kind", [("tiny", 1), ("tiny", 2), ("qc2640", 2), ("qc2640", 3)])
def test_orbit_reduced_patterns(ctx, oracle_mod, name, kind):
    import paper_2208_05795_amd as tsg
    code = {"tiny": workloads.tiny_code, "qc2640": workloads.qc2640_code}[name]()
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    full = oracle_mod.patterns(oc, kind)
    red = g.make_patterns(kind | tsg.PAT_QC_ORBITS)
    canon = {tuple(oracle_mod.canon(oc, p)[0]) for p in full}
    got = [tuple(int(x) for x in p) for p in red]
    _say(f"{name} kind {kind}: {len(full)} patterns -> {len(red)} orbit representatives (z = {code.z})")
    assert len(set(got)) == len(got)
    assert set(got) == canon
    assert len(red) * code.z >= len(full)
    g.free()


def test_orbit_reduction_rejects_csr(ctx):
    import paper_2208_05795_amd as tsg
    g = ctx.load_code(workloads.peg1008_code())
    with pytest.raises(tsg.TsgError):
        g.make_patterns(tsg.PAT_PAIRS | tsg.PAT_QC_ORBITS)
    g.free()


@pytest.mark.parametrize("name,decoder", [("tiny", 0), ("qc2640", 1)])
def test_orbit_reduced_search_finds_same_ts(ctx, name, decoder):
    import paper_2208_05795_amd as tsg
    code = {"tiny": workloads.tiny_code, "qc2640": workloads.qc2640_code}[name]()
    g = ctx.load_code(code)
    kinds = [1, 2] if name == "tiny" else [3]
    kw = dict(a_max=12) if decoder == 0 else dict(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024,
                                                   k_den=1024, a_max=12)
    full = g.pattern_list(kinds)
    red = g.pattern_list([k | tsg.PAT_QC_ORBITS for k in kinds])
    g.reset_ts()
    rf = g.impulse_search(full, **kw)
    ts_full = sorted(_ts_key(r) for r in g.collect())
    g.reset_ts()
    rr = g.impulse_search(red, **kw)
    ts_red = sorted(_ts_key(r) for r in g.collect())
    _say(f"{name} dec {decoder}: full {len(full)} patterns, {rf['stats']['decode_ms']:.1f} ms, "
         f"{len(ts_full)} TS; reduced {len(red)} patterns, {rr['stats']['decode_ms']:.1f} ms, "
         f"{len(ts_red)} TS")
    assert ts_full == ts_red
    # k* of each representative equals k* of its place in the full list
    index = {tuple(int(x) for x in p): i for i, p in enumerate(full)}
    kf = np.asarray(rf["k_crit"])
    kr = np.asarray(rr["k_crit"])
    for i, p in enumerate(red):
        assert kr[i] == kf[index[tuple(int(x) for x in p)]]
    g.free()


def test_spectrum_matches_oracle(ctx, oracle_mod, tiny, tiny_search):
    code, oc = tiny
    pats, ref = tiny_search
    g = ctx.load_code(code)
    g.impulse_search(pats, a_max=6)
    for by_orbit in (True, False):
        spec = g.spectrum(a_max=6, b_max=12, by_orbit=by_orbit)
        want = np.zeros_like(spec)
        for r in ref["ts"]:
            if r.b <= 12:
                want[r.a, r.b] += 1 if by_orbit else r.orbit
        assert np.array_equal(spec, want), by_orbit
    _say(f"tiny spectrum: {int(spec.sum())} sets; (a,b) cells {int((spec > 0).sum())}")
    g.free()


def test_union_bound_matches_oracle(ctx, oracle_mod, tiny, tiny_search):
    code, oc = tiny
    pats, ref = tiny_search
    g = ctx.load_code(code)
    g.impulse_search(pats, a_max=6)
    ts = g.collect()[:4]
    snrs = [2.0, 4.0]
    K = 2000
    ub = g.union_bound(len(ts), snrs, K, seed=21, shift=1.0, per_ts=True)
    for si, snr in enumerate(snrs):
        fer, var = 0.0, 0.0
        for t, r in enumerate(ts):
            o = oracle_mod.is_estimate(oc, list(r.bits), snr, 1.0, K, seed=21, stream=(si << 16) | t)
            fer += r.orbit * o["p_hat"]
            var += r.orbit ** 2 * o["var"]
            assert ub["per_ts"][si][t]["n"] == K
        p = ub["points"][si]
        half = 1.96 * np.sqrt(var)
        _say(f"union bound {snr} dB over {len(ts)} TS: gpu {p['fer']:.4e} oracle {fer:.4e} +- {half:.2e}")
        assert abs(p["fer"] - fer) <= max(0.02 * abs(fer), half)
    g.free()


def test_union_bound_validation(ctx, tiny):
    import paper_2208_05795_amd as tsg
    code, _ = tiny
    g = ctx.load_code(code)
    g.reset_ts()
    with pytest.raises(tsg.TsgError):   # empty table
        g.union_bound(1, [3.0], 100, seed=1)
    g.free()


def _table2():
    import os
    out = {}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "table2_code1_emd.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                L, emd, cnt = (int(x) for x in line)
                out[(L, emd)] = cnt
    return out


def test_cycle_emd_table2(ctx):
    """The library's chain walk reproduces Table II (Code 1, Table V): 4- and
    6-cycles exactly; 8-cycles at EMD 3..7 (Table II counts exponent chains,
    so its 8,2 entry is the girth-4 chain walked twice and its 8,8 entry rounds
    5380.5 orbits)."""
    g = ctx.load_code(workloads.table5_code1())
    out = g.cycle_emd(max_len=8, emd_max=16)
    tab = _table2()
    for L in (4, 6):
        half = L // 2
        got = {emd: out[half, emd] / half for emd in range(out.shape[1]) if out[half, emd]}
        want = {emd: float(cnt) for (l, emd), cnt in tab.items() if l == L}
        assert got == want, (L, got, want)
    got8 = {emd: out[4, emd] / 4 for emd in range(out.shape[1]) if out[4, emd]}
    for emd in range(3, 8):
        assert got8.get(emd, 0) == tab[(8, emd)], emd
    assert got8.get(2, 0) == 0 and got8[8] == 5380.5
    _say(f"Table II reproduced: {int(out.sum())} cycle incidences up to length 8")
    g.free()


@pytest.mark.parametrize("name,max_len", [("tiny", 8), ("qc2640", 10), ("batch", 8)])
def test_cycle_emd_matches_oracle(ctx, oracle_mod, name, max_len):
    code = {"tiny": workloads.tiny_code, "qc2640": workloads.qc2640_code,
            "batch": lambda: workloads.batch_codes()[3]}[name]()
    oc = oracle_mod.OCode(code)
    want, _, _ = oracle_mod.cycle_emd(oc, max_len=max_len, emd_max=24)
    g = ctx.load_code(code)
    got = g.cycle_emd(max_len=max_len, emd_max=24)
    assert np.array_equal(got, want)
    g.free()


def test_cycle_emd_rejects_csr(ctx):
    import paper_2208_05795_amd as tsg
    g = ctx.load_code(workloads.peg1008_code())
    with pytest.raises(tsg.TsgError):
        g.cycle_emd()
    g.free()
