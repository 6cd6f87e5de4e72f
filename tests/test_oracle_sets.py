"""Oracle pins: Tree(), TS(), (a,b) and the QC canonical form.

Pinned by hand-built graphs, by the structural a<=3 cells of Table III (Code 1),
by brute force and by the QC shift automorphism (abstract, Section II).
"""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def hexagon(oracle_mod):
    """v0-c0-v1-c1-v2-c2-v0 (a 6-cycle) with a private check on each variable,
    plus v3 joined to c0 only and v4 joined to c0 and c1."""
    rows = [[0, 1, 3, 4], [1, 2, 4], [0, 2], [0], [1], [2], [3], [4]]
    rp = np.cumsum([0] + [len(r) for r in rows])
    col = np.concatenate(rows)
    return oracle_mod.OCode(workloads.csr_code(5, len(rows), rp, col))


def test_ab_of_cycle(oracle_mod, hexagon):
    # the 6-cycle with one extra check per variable is TS(3,3)
    assert oracle_mod.count_b(hexagon, [0, 1, 2]) == 3
    assert list(oracle_mod.tree(hexagon, [0, 1, 2])) == [0, 1, 2]


def test_tree_drops_tree_like_parts(oracle_mod, hexagon):
    # a pair sharing one check is a tree: Tree() is empty
    assert oracle_mod.tree(hexagon, [0, 1]).size == 0
    # a pendant variable (v3 on c0 only) is peeled from the cycle
    assert list(oracle_mod.tree(hexagon, [0, 1, 2, 3])) == [0, 1, 2]
    # v4 shares c0 and c1 with the cycle: it stays
    assert list(oracle_mod.tree(hexagon, [0, 1, 2, 4])) == [0, 1, 2, 4]


def test_ts_closure_adds_cycle_closers(oracle_mod, hexagon):
    # {v0,v1}: v2 touches c1 and c2, both in the one component of G[{v0,v1}]; so
    # does v4 (c0, c1); v3 touches only c0
    assert list(oracle_mod.ts_closure(hexagon, [0, 1])) == [0, 1, 2, 4]
    # single pass: {v3} alone has one check, nobody closes a cycle with it
    assert list(oracle_mod.ts_closure(hexagon, [3])) == [3]
    # S2 for {v0,v1}: Tree(TS) = the cycle plus v4
    assert list(oracle_mod.tree(hexagon, oracle_mod.ts_closure(hexagon, [0, 1]))) == [0, 1, 2, 4]


def test_ts_closure_needs_same_component(oracle_mod):
    """u touching two checks of two different components is not added."""
    # c0 = {v0, v2}, c1 = {v1, v2}, c2={v0}, c3={v1}: G[{v0,v1}] has two components
    rows = [[0, 2], [1, 2], [0], [1], [2]]
    rp = np.cumsum([0] + [len(r) for r in rows])
    oc = oracle_mod.OCode(workloads.csr_code(3, 5, rp, np.concatenate(rows)))
    assert list(oracle_mod.ts_closure(oc, [0, 1])) == [0, 1]


def test_table3_structural_cells(oracle_mod, code1):
    """Table III prints TS(2,2) = TS(3,2) = 128 for Code 1: one full QC orbit each.
    Brute force over every connected set with a <= 3 that is its own 2-core finds
    exactly one orbit of 128 sets in each of these cells."""
    c, oc = code1
    n, counts, orbits = oracle_mod.brute_ts(oc, 3, 12)
    with open(os.path.join(GOLDEN, "table3_code1_small.txt")) as f:
        for line in f:
            t = line.split("#", 1)[0].split()
            if t:
                a, b, cnt = (int(x) for x in t)
                assert counts[a, b] == cnt and orbits[a, b] == 1
    # b = 2 is the smallest b for a <= 3, and a = 2 only has the 4-cycle
    assert counts[2].sum() == 128 and counts[3, :2].sum() == 0


def test_brute_sets_recount(oracle_mod, tiny):
    c, oc = tiny
    lst = oracle_mod.brute_ts_list(oc, 4)
    assert len(lst) > 0
    for a, b, s in lst:
        assert len(s) == a
        assert oracle_mod.count_b(oc, s) == b
        assert tuple(oracle_mod.tree(oc, s)) == s
        cs, orbit = oracle_mod.canon(oc, s)
        assert tuple(cs) == s and 16 % orbit == 0


def test_canon_shift_invariance(oracle_mod, tiny):
    c, oc = tiny
    z = c.z
    rng = np.random.default_rng(7)
    for _ in range(40):
        k = int(rng.integers(1, 8))
        s = np.sort(rng.choice(oc.n, size=k, replace=False)).astype(np.int32)
        cs, orbit = oracle_mod.canon(oc, s)
        images = set()
        for t in range(z):
            img = np.sort((s // z) * z + (s % z + t) % z)
            images.add(tuple(img))
            ci, oi = oracle_mod.canon(oc, img)
            assert tuple(ci) == tuple(cs) and oi == orbit
        assert tuple(cs) == min(images)
        assert len(images) == orbit   # orbit-stabiliser: |orbit| = z / |stab|


def test_canon_non_qc_is_sorted_set(oracle_mod):
    c = workloads.peg1008_code()
    oc = oracle_mod.OCode(c)
    s, orbit = oracle_mod.canon(oc, [500, 3, 77])
    assert list(s) == [3, 77, 500] and orbit == 1


def test_canon_stabilised_set(oracle_mod, tiny):
    """A set fixed by the half-turn t = z/2 has orbit z/2."""
    c, oc = tiny
    s = [0, 8]
    cs, orbit = oracle_mod.canon(oc, s)
    assert orbit == 8 and list(cs) == [0, 8]
