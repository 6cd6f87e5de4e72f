"""Oracle pins for the impulse search (Section III).

* every emitted TS recounts to its (a,b) and is its own Tree();
* the search finds every smallest trapping set that brute force enumerates;
* its (a,0) sets reproduce the exact minimum distance (Gray code);
* the whole search commutes with the QC shift automorphism.
"""
from collections import Counter

import numpy as np
import pytest

import workloads


def test_patterns_tiny(oracle_mod, tiny):
    c, oc = tiny
    s = oracle_mod.patterns(oc, oracle_mod.PAT_SINGLES)
    assert s.shape == (96, 1) and (s[:, 0] == np.arange(96)).all()
    p = oracle_mod.patterns(oc, oracle_mod.PAT_PAIRS)
    # every variable has 15 variables at distance 2 (girth 6, dv=3, dc=6)
    rp, col = oc.csr()
    nb2 = [set() for _ in range(oc.n)]
    for r in range(oc.m):
        vs = col[rp[r]:rp[r + 1]]
        for u in vs:
            nb2[u].update(int(v) for v in vs if v != u)
    assert all(len(x) == 15 for x in nb2)
    want = set()
    for u in range(oc.n):
        d4 = set(nb2[u])
        for w in nb2[u]:
            d4 |= nb2[w]
        d4.discard(u)
        want |= {(min(u, v), max(u, v)) for v in d4}
    assert set(map(tuple, p.tolist())) == want
    assert (np.diff(p[:, 0]) >= 0).all()
    t = oracle_mod.patterns(oc, oracle_mod.PAT_TRIPLES)
    assert (t[:, 0] < t[:, 1]).all() and (t[:, 1] < t[:, 2]).all()
    # 96 roots * 15 second variables * 10 third variables / 2 directions, except
    # that the three variables of a 6-cycle are reached through three middles
    n6 = oracle_mod.brute_ts(oc, 3, 12)[1][3].sum()
    assert len(t) == 96 * 15 * 10 // 2 - 2 * n6


def test_search_outputs_consistent(oracle_mod, tiny, tiny_search):
    c, oc = tiny
    pats, res = tiny_search
    kc, ic, il = res["k_crit"], res["iters_crit"], res["iters_lo"]
    assert ((kc == -1) | ((kc >= 1) & (kc <= 512))).all()
    fails = kc >= 0
    assert ((ic[fails] >= 1) & (ic[fails] <= 20)).all()
    assert ((il >= 1) & (il <= 20)).all()
    # decodes = 1 for patterns that never fail, 1 + 9 for the others
    assert res["decodes"] == int((~fails).sum()) + 10 * int(fails.sum())
    # re-decoding a pattern at k* fails and at k*-1 succeeds
    qb = oracle_mod.q_base(3.0, 0.5)
    rng = np.random.default_rng(3)
    for p in rng.choice(np.nonzero(fails)[0], 25, replace=False):
        for k, want in ((kc[p], 1), (kc[p] - 1, 0)):
            q = np.full(oc.n, qb)
            for v in pats[p]:
                if v >= 0:
                    q[v] = oracle_mod.q_impulse(qb, int(k))
            r = oracle_mod.decode_oms(oc, q, 20, 1)
            assert r["fail"] == want or (k == 0 and want == 0)
            if want:
                assert r["iters"] == ic[p]


def test_emitted_sets_are_trapping_sets(oracle_mod, tiny, tiny_search):
    """Definition check (Section II) on 100% of the emitted sets."""
    c, oc = tiny
    _, res = tiny_search
    assert len(res["ts"]) > 0
    seen = set()
    for r in res["ts"]:
        assert 1 <= r.a <= 6 and len(r.bits) == r.a
        assert oracle_mod.count_b(oc, r.bits) == r.b
        assert tuple(oracle_mod.tree(oc, r.bits)) == r.bits
        cs, orbit = oracle_mod.canon(oc, r.bits)
        assert tuple(cs) == r.bits and orbit == r.orbit
        assert r.bits not in seen
        seen.add(r.bits)
    # total order: b/a, then a, then the tuple
    keys = [(r.b / r.a, r.a, r.bits) for r in res["ts"]]
    assert keys == sorted(keys)


def _recall(oracle_mod, oc, res, a_max=6):
    brute = oracle_mod.brute_ts_list(oc, a_max)
    found = {r.bits for r in res["ts"]}
    by_cell = Counter((a, b) for a, b, _ in brute)
    hit = Counter((a, b) for a, b, s in brute if s in found)
    return brute, by_cell, hit


def test_search_recall_smallest_sets(oracle_mod, tiny, tiny_search):
    """Brute force over all connected TS with a <= 6 (orbits of the QC shift),
    against the search over the tiny code's singles and pairs within distance 4.
    Full recall of every cell with a <= 4, including the minimum-a cell (3,3)
    and the (4,0) codeword.  The other cells with b <= a are reported; the
    recall there is a property of the heuristic's pattern set (measured: (5,3)
    41/42, (6,2) 12/13, (5,5) 255/598, (6,4) 236/1334, (6,6) 267/5260), and is
    held to those counts as a floor."""
    c, oc = tiny
    _, res = tiny_search
    brute, by_cell, hit = _recall(oracle_mod, oc, res)
    print("\nrecall, singles + pairs: " + ", ".join(
        f"({a},{b}) {hit[(a, b)]}/{n}" for (a, b), n in sorted(by_cell.items()) if b <= a))
    a_min = min(a for a, _ in by_cell)
    assert a_min == 3
    for (a, b), n in by_cell.items():
        if a <= 4:
            assert hit[(a, b)] == n, ((a, b), hit[(a, b)], n)
    floor = {(5, 3): 41, (6, 2): 12, (5, 5): 255, (6, 4): 236, (6, 6): 267}
    for cell, k in floor.items():
        assert hit[cell] >= k, (cell, hit[cell], by_cell[cell])
    # every connected emitted set is one of the brute-force sets
    brute_set = {s for _, _, s in brute}
    adj = _var_adjacency(oc)
    for r in res["ts"]:
        if _connected(r.bits, adj):
            assert r.bits in brute_set


def test_search_recall_with_triples(oracle_mod, tiny):
    """Adding the tree-path triples of the impulse tree (Section III, Fig. 3)
    recovers the (5,3) and (6,2) orbits that singles and pairs miss: every cell
    with b/a < 1 and a <= 6 except (6,4) is then complete."""
    c, oc = tiny
    pats = oracle_mod.pattern_list(oc, [1, 2, 3])
    res = oracle_mod.search(oc, pats, a_max=6)
    _, by_cell, hit = _recall(oracle_mod, oc, res)
    print("\nrecall, singles + pairs + triples: " + ", ".join(
        f"({a},{b}) {hit[(a, b)]}/{n}" for (a, b), n in sorted(by_cell.items()) if b <= a))
    for cell in ((3, 3), (4, 0), (4, 2), (4, 4), (5, 3), (6, 2)):
        assert hit[cell] == by_cell[cell], (cell, hit[cell], by_cell[cell])
    floor = {(5, 5): 422, (6, 4): 570, (6, 6): 613}
    for cell, k in floor.items():
        assert hit[cell] >= k, (cell, hit[cell], by_cell[cell])


def _var_adjacency(oc):
    rp, col = oc.csr()
    adj = [set() for _ in range(oc.n)]
    for r in range(oc.m):
        vs = [int(v) for v in col[rp[r]:rp[r + 1]]]
        for u in vs:
            adj[u].update(v for v in vs if v != u)
    return adj


def _connected(s, adj):
    s = set(s)
    start = next(iter(s))
    seen = {start}
    stack = [start]
    while stack:
        u = stack.pop()
        for v in adj[u] & s:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return seen == s


def test_dmin_equals_smallest_codeword_ts(oracle_mod):
    """Section II: TS(d_min, 0) are the minimum-weight codewords.  On the Z=8
    variant (dimension small enough for Gray-code enumeration) the exact d_min,
    the brute-force smallest (a,0) set and the search's smallest (a,0) set agree."""
    c = workloads.tiny_code_z8()
    oc = oracle_mod.OCode(c)
    d, word = oracle_mod.dmin(oc)
    assert oracle_mod.count_b(oc, word) == 0 and len(word) == d
    n, counts, _ = oracle_mod.brute_ts(oc, 6, 12)
    a0 = [a for a in range(7) if counts[a, 0]]
    assert a0 and a0[0] == d
    pats = oracle_mod.pattern_list(oc, [oracle_mod.PAT_SINGLES, oracle_mod.PAT_PAIRS])
    res = oracle_mod.search(oc, pats, a_max=8)
    cw = [r.a for r in res["ts"] if r.b == 0]
    assert cw and min(cw) == d


def test_dmin_tiny_code(oracle_mod, tiny, tiny_search):
    """A minimum-weight codeword's support is connected and its own 2-core, so the
    brute-force (a <= 6) list holds every codeword of weight <= 6."""
    c, oc = tiny
    n, counts, orbits = oracle_mod.brute_ts(oc, 6, 12)
    assert counts[4, 0] == 16 and orbits[4, 0] == 1 and counts[:4, 0].sum() == 0
    _, res = tiny_search
    assert [r.a for r in res["ts"] if r.b == 0] == [4]


@pytest.mark.parametrize("t", [1, 5, 11])
def test_search_commutes_with_qc_shift(oracle_mod, tiny, tiny_search, t):
    """QC automorphism: the search on sigma_t(patterns) gives identical k*,
    iteration counts and the same canonical TS list."""
    c, oc = tiny
    pats, res = tiny_search
    z = c.z
    sp = np.where(pats >= 0, (pats // z) * z + (pats % z + t) % z, -1).astype(np.int32)
    r2 = oracle_mod.search(oc, sp, a_max=6)
    for key in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand"):
        assert (r2[key] == res[key]).all(), key
    a = [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in res["ts"]]
    b = [(r.a, r.b, r.orbit, r.k_crit, r.bits) for r in r2["ts"]]
    assert a == b


def test_extract_critical_is_subset(oracle_mod, tiny, tiny_search):
    c, oc = tiny
    pats, res = tiny_search
    r2 = oracle_mod.search(oc, pats, a_max=6, extract_mode=oracle_mod.EXTRACT_CRITICAL)
    assert (r2["k_crit"] == res["k_crit"]).all()
    assert (r2["n_cand"] <= res["n_cand"]).all()
    assert {r.bits for r in r2["ts"]} <= {r.bits for r in res["ts"]}


def test_spa_search_small(oracle_mod, tiny):
    c, oc = tiny
    pats = oracle_mod.patterns(oc, oracle_mod.PAT_PAIRS)[:200]
    res = oracle_mod.search(oc, pats, decoder=oracle_mod.DEC_SPA, max_iter=50,
                            k_max=32 * 1024, k_den=1024, a_max=6)
    kc = res["k_crit"]
    assert ((kc == -1) | (kc >= 1)).all()
    assert res["decodes"] == int((kc < 0).sum()) + 16 * int((kc >= 0).sum())
    for r in res["ts"]:
        assert oracle_mod.count_b(oc, r.bits) == r.b
    # the bisection's transition: re-decoding a pattern at k* fails (with the
    # reported iteration count and minimum-syndrome iteration) and at k* - 1
    # succeeds
    h = 2.0 / oracle_mod.sigma2(3.0, 0.5)
    rng = np.random.default_rng(6)
    fails = np.nonzero(kc >= 0)[0]
    assert len(fails) >= 25
    for p in rng.choice(fails, 25, replace=False):
        for k, want in ((kc[p], 1), (kc[p] - 1, 0)):
            llr = np.full(oc.n, h)
            for v in pats[p]:
                llr[v] = h * (1.0 - k / 1024.0)
            r = oracle_mod.decode_spa(oc, llr, 50)
            assert r["fail"] == want, (p, k)
            if want:
                assert r["iters"] == res["iters_crit"][p] and r["tmin"] == res["tmin_crit"][p]


def test_spa_eps_star_is_a_transition(oracle_mod, tiny, tiny_search):
    """eps* of an impulse on a whole set (the IS shift of Section I/II): the SPA
    decode fails at eps* and succeeds one grid step (2^-10) below."""
    c, oc = tiny
    _, res = tiny_search
    h = 2.0 / oracle_mod.sigma2(3.0, 0.5)
    sets = [r.bits for r in res["ts"] if r.a >= 3][:6]
    for bits in sets:
        eps = oracle_mod.spa_eps_star(oc, bits, 3.0)
        assert eps > 0
        for e, want in ((eps, 1), (eps - 1.0 / 1024.0, 0)):
            llr = np.full(oc.n, h)
            llr[list(bits)] = h * (1.0 - e)
            assert oracle_mod.decode_spa(oc, llr, 50)["fail"] == want, (bits, e)


def test_lnms_search_consistent(oracle_mod, tiny):
    """Layered min-sum search: re-decoding at k* fails and at k*-1 succeeds,
    every emitted set recounts, and the search commutes with the QC shift."""
    c, oc = tiny
    pats = oracle_mod.pattern_list(oc, [1, 2])
    kw = dict(decoder=oracle_mod.DEC_LNMS, llr_scale=1.0, a_max=6)
    res = oracle_mod.search(oc, pats, **kw)
    kc = res["k_crit"]
    fails = kc >= 0
    assert fails.any()
    qb = oracle_mod.q4_base(3.0, 0.5, 1.0)
    rng = np.random.default_rng(4)
    for p in rng.choice(np.nonzero(fails)[0], 25, replace=False):
        for k, want in ((kc[p], 1), (kc[p] - 1, 0)):
            q = np.full(oc.n, qb)
            for v in pats[p]:
                if v >= 0:
                    q[v] = oracle_mod.q4_impulse(qb, int(k))
            assert oracle_mod.decode_lnms(oc, q, 20)["fail"] == want
    for r in res["ts"]:
        assert oracle_mod.count_b(oc, r.bits) == r.b
        assert tuple(oracle_mod.tree(oc, r.bits)) == r.bits
    sp = np.where(pats >= 0, (pats // c.z) * c.z + (pats % c.z + 5) % c.z, -1).astype(np.int32)
    r2 = oracle_mod.search(oc, sp, **kw)
    assert (r2["k_crit"] == kc).all()
    assert [x.bits for x in r2["ts"]] == [x.bits for x in res["ts"]]
