"""Oracle pins: QC expansion and girth against the paper's printed Code 1.

Code 1 is the 4x20, L=128 exponent matrix of Table V.  Expanding it with the
circulant convention of Section II (P^k: row r has its one in column (r+k) mod L)
must reproduce the cycle/EMD spectrum of Table II column "Code 1" and the
per-row / per-column cycle averages of Table V.  A wrong circulant direction, a
transposed block or an off-by-one shift changes these counts.
"""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table2():
    out = {}
    with open(os.path.join(GOLDEN, "table2_code1_emd.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                L, emd, cnt = (int(x) for x in line)
                out[(L, emd)] = cnt
    return out


def _table5_rows():
    rows = {}
    with open(os.path.join(GOLDEN, "table5_code1.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line and line[0] != "E":
                rows[line[0]] = [int(x) for x in line[1:]]
    return rows


def test_code1_shape(code1):
    c, oc = code1
    # "77 non-zero circulants" (Section III text), L = 128, 4 x 20 blocks
    assert int((c.shifts >= 0).sum()) == 77
    assert (oc.n, oc.m, oc.e) == (2560, 512, 77 * 128)
    # Table III caption: Code 1 has girth 4
    assert oc.girth == 4
    rp, col = oc.csr()
    colw = np.bincount(col, minlength=oc.n).reshape(20, 128)
    assert (colw == colw[:, :1]).all()
    assert list(colw[:, 0]) == [3, 3, 3] + [4] * 17


@pytest.fixture(scope="module")
def code1_cycles(oracle_mod, code1):
    return oracle_mod.cycle_emd(code1[1], max_len=8, emd_max=16)


def test_code1_table2_short_cycles(code1_cycles):
    """4- and 6-cycles per QC orbit and EMD equal Table II exactly."""
    out, _, _ = code1_cycles
    tab = _table2()
    for L in (4, 6):
        half = L // 2
        got = {emd: out[half, emd] / half for emd in range(out.shape[1]) if out[half, emd]}
        want = {emd: float(cnt) for (l, emd), cnt in tab.items() if l == L}
        assert got == want, (L, got, want)


def test_code1_table2_eight_cycles(code1_cycles):
    """8-cycles: EMD 3..7 equal Table II.  Table II counts exponent chains, so its
    '8,2 = 1' is the girth-4 chain walked twice (not a simple cycle) and its
    '8,8 = 5381' rounds 5378 full orbits plus 5 half-size orbits (= 5380.5)."""
    out, _, _ = code1_cycles
    tab = _table2()
    got = {emd: out[4, emd] / 4 for emd in range(out.shape[1]) if out[4, emd]}
    for emd in range(3, 8):
        assert got.get(emd, 0) == tab[(8, emd)], emd
    assert got.get(2, 0) == 0 and tab[(8, 2)] == 1
    assert got[8] == 5380.5 and tab[(8, 8)] == 5381


def test_code1_table5_row_column_averages(code1_cycles):
    """Table V: average number of 4/6-cycles through each block row / column,
    relative to 128 (the cycle count divided by its length / 2)."""
    _, per_row, per_col = code1_cycles
    rows = _table5_rows()
    assert list(per_row[2] // 2) == rows["CYC4ROW2"]
    assert list(per_row[3] // 3) == rows["CYC6ROW3"]
    assert list(per_col[2] // 2) == rows["CYC4COL2"]
    assert list(per_col[3] // 3) == rows["CYC6COL3"]
    assert (per_row[2] % 2 == 0).all() and (per_row[3] % 3 == 0).all()
    # the 163 six-cycle orbits are the sum of the row averages
    assert sum(rows["CYC6ROW3"]) == 3 * 163


def test_girth_hand_graphs(oracle_mod):
    # a 6-cycle v0-c0-v1-c1-v2-c2-v0 plus a private check on each variable
    rp = [0, 2, 4, 6, 7, 8, 9]
    col = [0, 1, 1, 2, 0, 2, 0, 1, 2]
    oc = oracle_mod.OCode(workloads.csr_code(3, 6, rp, col))
    assert oc.girth == 6
    # cycle-free: a path of checks
    oc = oracle_mod.OCode(workloads.csr_code(4, 3, [0, 2, 4, 6], [0, 1, 1, 2, 2, 3]))
    assert oc.girth == 0
    # a 4-cycle: two checks sharing two variables
    oc = oracle_mod.OCode(workloads.csr_code(3, 2, [0, 3, 5], [0, 1, 2, 0, 1]))
    assert oc.girth == 4


def test_qc_expansion_convention(oracle_mod):
    """Section II, eq. (1): P_ij = 1 iff i+1 = j (mod L), so P^1 row r -> column r+1."""
    oc = oracle_mod.OCode(workloads.qc_code([[1]], 5))
    rp, col = oc.csr()
    assert list(col) == [1, 2, 3, 4, 0]
    oc = oracle_mod.OCode(workloads.qc_code([[0, 3], [-1, 2]], 4))
    rp, col = oc.csr()
    rows = [sorted(col[rp[r]:rp[r + 1]]) for r in range(8)]
    assert rows[0] == [0, 4 + 3] and rows[1] == [1, 4 + 0]
    assert rows[4] == [4 + 2] and rows[6] == [4 + 0]


def test_generated_codes_meet_girth(oracle_mod):
    assert oracle_mod.OCode(workloads.tiny_code()).girth >= 6
    assert oracle_mod.OCode(workloads.tiny_code_z8()).girth >= 6
    assert oracle_mod.OCode(workloads.qc2640_code()).girth >= 8
    peg = oracle_mod.OCode(workloads.peg1008_code())
    assert peg.girth >= 6 and peg.e == 3024


def test_invalid_codes_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.OCode(workloads.csr_code(3, 1, [0, 2], [0, 0]))   # duplicate edge
    with pytest.raises(ValueError):
        oracle_mod.OCode(workloads.csr_code(3, 1, [0, 2], [0, 1]))   # empty column 2
