"""GPU parity of the quantised normalised layered min-sum (4/4/6 bits) impulse
search against the oracle: bit-exact critical amplitudes, iteration counts,
first minimum-syndrome iterations, candidate counts and the whole ordered TS
list, on a QC code (layers = block rows) and a PEG code (greedy layers)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")
LNMS = dict(k_max=512, k_den=16)


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


# (code, pattern kinds, sample, iterations, Eb/N0, channel scale): the first
# cases decode almost everything; the weaker channel scales and short
# iteration budgets give failing impulses, candidates and trapping sets
CASES = [("tiny", [1, 2], 0, 20, 3.0, 1.0), ("tiny", [1, 2], 0, 3, 3.0, 1.0),
         ("peg1008", [1, 2, 3], 600, 20, 3.0, 1.0), ("qc2640", [3], 400, 20, 3.0, 1.0),
         ("peg1008", [1, 2, 3], 600, 3, 3.0, 0.5), ("peg1008", [1, 2, 3], 600, 20, 3.0, 0.3),
         ("qc2640", [3], 600, 2, 3.0, 0.5), ("qc2640", [3], 600, 20, 3.0, 0.3)]


@pytest.mark.parametrize("name,kinds,sample,iters,snr,scale", CASES)
def test_lnms_search_bit_exact(ctx, oracle_mod, name, kinds, sample, iters, snr, scale):
    import paper_2208_05795_amd as tsg
    code = {"tiny": workloads.tiny_code, "peg1008": workloads.peg1008_code,
            "qc2640": workloads.qc2640_code}[name]()
    oc = oracle_mod.OCode(code)
    pats = oracle_mod.pattern_list(oc, kinds)
    if sample:
        rng = np.random.default_rng(61)
        pats = np.ascontiguousarray(pats[np.sort(rng.choice(len(pats), sample, replace=False))])
    kw = dict(max_iter=iters, ebn0_db=snr, llr_scale=scale, a_max=8, **LNMS)
    ref = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_LNMS, threads=8, **kw)
    g = ctx.load_code(code)
    got = g.impulse_search(pats, decoder=tsg.DEC_LNMS, **kw)
    for k in KEYS:
        if not np.array_equal(np.asarray(got[k]), ref[k]):
            bad = np.nonzero(np.asarray(got[k]) != ref[k])[0]
            raise AssertionError(f"{k} differs at {bad[:8]}: {np.asarray(got[k])[bad[:8]]} vs {ref[k][bad[:8]]}")
    assert _ts(g.collect()) == _ts(ref["ts"])
    # the oracle computes every iteration; the fixed-point exit computes fewer
    assert got["stats"]["edge_updates"] <= ref["edge_updates"]
    full = g.impulse_search(pats, decoder=tsg.DEC_LNMS, full_iterations=True, **kw)
    assert full["stats"]["edge_updates"] == ref["edge_updates"]
    _say(f"{name} layered min-sum, {len(pats)} patterns, {iters} it, {snr} dB x {scale}: bit-exact; "
         f"{(ref['k_crit'] >= 0).sum()} failing, {int(ref['n_cand'].sum())} candidates, "
         f"{len(ref['ts'])} TS")
    g.free()


def test_lnms_rejects_bad_options(ctx):
    import paper_2208_05795_amd as tsg
    g = ctx.load_code(workloads.tiny_code())
    with pytest.raises(tsg.TsgError):
        g.impulse_search(np.array([[0]], dtype=np.int32), decoder=tsg.DEC_LNMS, k_den=1024)
    with pytest.raises(tsg.TsgError):   # no streamed form of the layered decoder
        g.impulse_search(np.array([[0]], dtype=np.int32), decoder=tsg.DEC_LNMS, llr_scale=1.0,
                         layout=tsg.LAYOUT_STREAMED)
    g.free()


@pytest.mark.parametrize("name", ["tiny", "peg1008", "qc2640"])
def test_layer_count_matches_oracle(ctx, oracle_mod, name):
    code = {"tiny": workloads.tiny_code, "peg1008": workloads.peg1008_code,
            "qc2640": workloads.qc2640_code}[name]()
    n_layers, _ = oracle_mod.layers(oracle_mod.OCode(code))
    g = ctx.load_code(code)
    assert g.info["n_layers"] == n_layers
    g.free()
