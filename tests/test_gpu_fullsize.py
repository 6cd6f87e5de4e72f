"""Full-size jobs in the launch configuration bench.py times, checked on sampled
outputs that the oracle recomputes one pattern at a time, and on properties
that hold at any size (every TS recounted against the definition, canonical,
its own Tree(), smallest producing pattern consistent with the sample).

PEG-1008 job: every single, pair (distance <= 4) and tree-path triple, OMS int8
(20 iterations) and SPA float32 (50 iterations), a_max = 12, 3 dB.
QC-2640 job: every tree-path triple, SPA float32 (50 iterations), a_max = 12.
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


def _check_ts_definitions(oracle_mod, oc, recs, a_max, z):
    for r in recs:
        assert 1 <= r.a <= a_max and len(r.bits) == r.a
        assert oracle_mod.count_b(oc, r.bits) == r.b
        assert tuple(oracle_mod.tree(oc, r.bits)) == r.bits
        cs, orbit = oracle_mod.canon(oc, r.bits)
        assert tuple(cs) == r.bits and orbit == r.orbit
    keys = [(r.b * 1.0 / r.a, r.a, r.bits) for r in recs]
    assert keys == sorted(keys)


def _sample_subset_check(ref, recs, idx):
    """TS the oracle finds from the sampled patterns are in the full list, with a
    first pattern no later and a k* no larger than the sample's."""
    full = {r.bits: r for r in recs}
    for r in ref["ts"]:
        g = full.get(r.bits)
        assert g is not None, r.bits
        assert g.first_pattern <= idx[r.first_pattern]
        assert g.k_crit <= r.k_crit


@pytest.fixture(scope="module")
def peg():
    return workloads.peg1008_code()


def test_peg1008_full_oms(ctx, oracle_mod, peg):
    import paper_2208_05795_amd as tsg
    import torch
    oc = oracle_mod.OCode(peg)
    g = ctx.load_code(peg)
    pats = g.pattern_list([1, 2, 3])
    _say(f"peg1008 full OMS job, {len(pats)} patterns")
    got = g.impulse_search(torch.from_numpy(pats).cuda(), a_max=12)
    recs = g.collect()
    got = {k: v.cpu().numpy() for k, v in got.items() if k != "stats"}
    rng = np.random.default_rng(31)
    idx = np.sort(rng.choice(len(pats), 600, replace=False))
    # make sure patterns that fail are represented
    fails = np.nonzero(got["k_crit"] >= 0)[0]
    if len(fails):
        idx = np.unique(np.concatenate([idx, rng.choice(fails, min(200, len(fails)), replace=False)]))
    ref = oracle_mod.search(oc, np.ascontiguousarray(pats[idx]), a_max=12)
    for k in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand"):
        assert np.array_equal(got[k][idx], ref[k]), k
    _check_ts_definitions(oracle_mod, oc, recs, 12, 0)
    _sample_subset_check(ref, recs, idx)
    g.free()


def test_peg1008_full_spa(ctx, oracle_mod, peg):
    import paper_2208_05795_amd as tsg
    import torch
    oc = oracle_mod.OCode(peg)
    g = ctx.load_code(peg)
    pats = g.pattern_list([1, 2, 3])
    _say(f"peg1008 full SPA job, {len(pats)} patterns")
    got = g.impulse_search(torch.from_numpy(pats).cuda(), decoder=tsg.DEC_SPA, max_iter=50,
                           k_max=32 * 1024, k_den=1024, a_max=12)
    recs = g.collect()
    kc = got["k_crit"].cpu().numpy()
    rng = np.random.default_rng(32)
    fails = np.nonzero(kc >= 0)[0]
    idx = np.unique(np.concatenate([rng.choice(len(pats), 60, replace=False),
                                    rng.choice(fails, min(60, len(fails)), replace=False)]))
    ref = oracle_mod.search(oc, np.ascontiguousarray(pats[idx]), decoder=oracle_mod.DEC_SPA,
                            max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12)
    ko = ref["k_crit"]
    kg = kc[idx]
    ok = ((kg == -1) & (ko == -1)) | ((kg >= 0) & (ko >= 0) & (np.abs(kg - ko) <= 1e-3 * np.maximum(ko, 1)))
    _say(f"  eps* within 1e-3 on {int(ok.sum())}/{len(ok)}, exact {int((kg == ko).sum())}")
    assert ok.all()
    _check_ts_definitions(oracle_mod, oc, recs, 12, 0)
    assert len(recs) > 100
    g.free()


def test_qc2640_full_spa_triples(ctx, oracle_mod):
    import paper_2208_05795_amd as tsg
    import torch
    code = workloads.qc2640_code()
    oc = oracle_mod.OCode(code)
    g = ctx.load_code(code)
    pats = g.make_patterns(3)
    _say(f"qc2640 full SPA triples job, {len(pats)} patterns")
    got = g.impulse_search(torch.from_numpy(pats).cuda(), decoder=tsg.DEC_SPA, max_iter=50,
                           k_max=32 * 1024, k_den=1024, a_max=12)
    recs = g.collect()
    st = got["stats"]
    _say(f"  {st['edge_updates']:.3e} edge-updates in {st['decode_ms']:.1f} ms; {len(recs)} TS")
    kc = got["k_crit"].cpu().numpy()
    rng = np.random.default_rng(33)
    fails = np.nonzero(kc >= 0)[0]
    idx = np.unique(np.concatenate([rng.choice(len(pats), 24, replace=False),
                                    rng.choice(fails, min(24, len(fails)), replace=False)]))
    ref = oracle_mod.search(oc, np.ascontiguousarray(pats[idx]), decoder=oracle_mod.DEC_SPA,
                            max_iter=50, k_max=32 * 1024, k_den=1024, a_max=12)
    ko, kg = ref["k_crit"], kc[idx]
    ok = ((kg == -1) & (ko == -1)) | ((kg >= 0) & (ko >= 0) & (np.abs(kg - ko) <= 1e-3 * np.maximum(ko, 1)))
    _say(f"  eps* within 1e-3 on {int(ok.sum())}/{len(ok)}, exact {int((kg == ko).sum())}")
    assert ok.all()
    _check_ts_definitions(oracle_mod, oc, recs, 12, code.z)
    # QC symmetry of the job: the pattern list is shift-closed, so every TS
    # orbit found is found whole: orbit sizes divide z
    assert all(code.z % r.orbit == 0 for r in recs)
    g.free()
