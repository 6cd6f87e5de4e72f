"""Seeded LDPC parity-check matrices shaped like the paper's test codes.

The paper's own codes (MacKay's PEG(1008,504), the Margulis (2640,1320) code and
Codes 2-5 of Section III) are not available, so these generators build stand-ins
with the same length, rate, degrees and girth.  Only Code 1, whose exponent
matrix the paper prints in Table V, is the paper's own.

A code is handed over in one of the two forms the library and the oracle accept:

* QC form: an ``mb x nb`` exponent matrix ``shifts`` (``-1`` = zero block, the
  paper's P^inf of Section II) and the circulant size ``z``;
* CSR form: ``row_ptr[m+1]`` / ``col[nnz]`` of H, rows = checks.

Neither side receives an expanded matrix from here; each expands QC form itself.

Cycle rejection during sampling uses the exponent-chain condition of
Proposition 1 (Section II): a closed non-backtracking walk of length 2l in the
base graph lifts to 2l-cycles iff its alternating exponent sum is 0 mod z.
"""
from __future__ import annotations

import dataclasses
import os
from typing import List, Optional

import numpy as np

_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "tests", "golden")


@dataclasses.dataclass
class Code:
    """A parity-check matrix in QC or CSR form (see module docstring)."""

    kind: str                      # "qc" or "csr"
    n: int                         # variable nodes (columns of H)
    m: int                         # check nodes (rows of H)
    name: str = ""
    mb: int = 0
    nb: int = 0
    z: int = 0
    shifts: Optional[np.ndarray] = None   # int32 [mb, nb], -1 = zero block
    row_ptr: Optional[np.ndarray] = None  # int64 [m+1]
    col: Optional[np.ndarray] = None      # int32 [nnz]

    @property
    def nnz(self) -> int:
        if self.kind == "qc":
            return int((self.shifts >= 0).sum()) * self.z
        return int(self.row_ptr[-1])

    @property
    def rate(self) -> float:
        """Design rate 1 - m/n (the rate the paper's sigma formula uses)."""
        return 1.0 - self.m / self.n


def qc_code(shifts, z: int, name: str = "") -> Code:
    s = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32))
    mb, nb = s.shape
    if np.any((s < -1) | (s >= z)):
        raise ValueError("shift out of range")
    return Code("qc", nb * z, mb * z, name, mb, nb, z, s)


def csr_code(n: int, m: int, row_ptr, col, name: str = "") -> Code:
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    c = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    return Code("csr", n, m, name, row_ptr=rp, col=c)


# ----------------------------------------------------------------------------
# exponent-chain cycle test on the base matrix (Proposition 1)
# ----------------------------------------------------------------------------

def _has_short_chain(s: np.ndarray, z: int, half_len: int) -> bool:
    """True iff some closed non-backtracking base walk of length 2*half_len has
    an alternating exponent sum of 0 mod z (i.e. H has a 2*half_len cycle)."""
    mb, nb = s.shape
    rows_of = [[i for i in range(mb) if s[i, j] >= 0] for j in range(nb)]
    cols_of = [[j for j in range(nb) if s[i, j] >= 0] for i in range(mb)]
    for i0 in range(mb):
        for j0 in cols_of[i0]:
            a = int(s[i0, j0])
            for i1 in rows_of[j0]:
                if i1 == i0:
                    continue
                acc = a - int(s[i1, j0])
                if _walk_rest(s, z, rows_of, cols_of, i0, j0, i1, j0, 1, half_len, acc):
                    return True
    return False


def _walk_rest(s, z, rows_of, cols_of, i0, j0, i, j, depth, half_len, acc):
    for j2 in cols_of[i]:
        if j2 == j:
            continue
        a1 = acc + int(s[i, j2])
        for i2 in rows_of[j2]:
            if i2 == i:
                continue
            a2 = a1 - int(s[i2, j2])
            if depth + 1 == half_len:
                if i2 == i0 and j2 != j0 and a2 % z == 0:
                    return True
            elif _walk_rest(s, z, rows_of, cols_of, i0, j0, i2, j2, depth + 1, half_len, a2):
                return True
    return False


def _girth_at_least(s: np.ndarray, z: int, g: int) -> bool:
    for half in range(2, (g + 1) // 2):
        if 2 * half >= g:
            break
        if _has_short_chain(s, z, half):
            return False
    return True


def qc_random_shifts(mb: int, nb: int, z: int, seed: int, girth_min: int,
                     max_draws: int = 1_000_000) -> np.ndarray:
    """All blocks nonzero, shifts i.i.d. U[0, z), redrawn until girth >= girth_min."""
    rng = np.random.default_rng(seed)
    for _ in range(max_draws):
        s = rng.integers(0, z, size=(mb, nb), dtype=np.int64).astype(np.int32)
        if _girth_at_least(s, z, girth_min):
            return s
    raise RuntimeError("no shift draw met the girth bound")


def qc_greedy_shifts(mask: np.ndarray, z: int, rng: np.random.Generator,
                     restarts: int = 20) -> Optional[np.ndarray]:
    """Column-by-column random shift assignment that never closes a 4-cycle.

    ``mask`` is the base matrix support.  Returns None when every restart got
    stuck (the caller then redraws z).
    """
    mb, nb = mask.shape
    for _ in range(restarts):
        s = np.full((mb, nb), -1, dtype=np.int32)
        ok = True
        for j in range(nb):
            rows = np.nonzero(mask[:, j])[0]
            rng.shuffle(rows)
            for idx, i in enumerate(rows):
                banned = np.zeros(z, dtype=bool)
                for i2 in rows[:idx]:
                    for j2 in range(j):
                        if s[i, j2] >= 0 and s[i2, j2] >= 0:
                            # 4-cycle iff s[i,j]-s[i2,j] == s[i,j2]-s[i2,j2] (mod z)
                            banned[(int(s[i2, j]) + int(s[i, j2]) - int(s[i2, j2])) % z] = True
                free = np.nonzero(~banned)[0]
                if free.size == 0:
                    ok = False
                    break
                s[i, j] = int(free[rng.integers(0, free.size)])
            if not ok:
                break
        if ok:
            return s
    return None


# ----------------------------------------------------------------------------
# progressive edge growth (Hu, Eleftheriou, Arnold), regular check degree
# ----------------------------------------------------------------------------

def peg_regular(n: int, m: int, dv: int, dc: int, seed: int) -> Code:
    """PEG construction with every check capped at degree dc (so n*dv == m*dc
    gives a (dv, dc)-regular H).  Each new edge of a variable goes to a
    lowest-degree check outside the variable's current depth-l neighbourhood,
    l as large as possible; ties are broken by the seeded generator."""
    if n * dv != m * dc:
        raise ValueError("n*dv must equal m*dc")
    rng = np.random.default_rng(seed)
    vadj: List[List[int]] = [[] for _ in range(n)]
    cadj: List[List[int]] = [[] for _ in range(m)]
    cdeg = np.zeros(m, dtype=np.int64)

    def pick(cands: np.ndarray) -> int:
        d = cdeg[cands]
        best = cands[d == d.min()]
        return int(best[rng.integers(0, best.size)])

    for v in range(n):
        for k in range(dv):
            open_c = cdeg < dc
            open_c[vadj[v]] = False
            if k == 0:
                cands = np.nonzero(open_c)[0]
            else:
                reached = np.zeros(m, dtype=bool)
                seen_v = np.zeros(n, dtype=bool)
                seen_v[v] = True
                frontier_v = [v]
                prev_layer = None
                while True:
                    new_c = []
                    for u in frontier_v:
                        for c in vadj[u]:
                            if not reached[c]:
                                reached[c] = True
                                new_c.append(c)
                    avail_unreached = open_c & ~reached
                    if not avail_unreached.any():
                        # every open check is within reach: take the deepest layer
                        layer = np.array(new_c if new_c else (prev_layer or []), dtype=np.int64)
                        layer = layer[open_c[layer]] if layer.size else layer
                        cands = layer if layer.size else np.nonzero(open_c)[0]
                        break
                    if not new_c:
                        cands = np.nonzero(avail_unreached)[0]
                        break
                    prev_layer = new_c
                    nxt = []
                    for c in new_c:
                        for u in cadj[c]:
                            if not seen_v[u]:
                                seen_v[u] = True
                                nxt.append(u)
                    frontier_v = nxt
            c = pick(cands)
            vadj[v].append(c)
            cadj[c].append(v)
            cdeg[c] += 1
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(a) for a in cadj])
    col = np.concatenate([np.sort(np.array(a, dtype=np.int32)) for a in cadj])
    return csr_code(n, m, row_ptr, col, name=f"peg{n}x{m}-s{seed}")


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def tiny_code() -> Code:
    """3x6 base, Z=16 (N=96, M=48, 288 edges), seed 1, girth >= 6."""
    return qc_code(qc_random_shifts(3, 6, 16, seed=1, girth_min=6), 16, "tiny-qc96")


def tiny_code_z8() -> Code:
    """3x6 base, Z=8 (N=48): small enough for an exact minimum distance."""
    return qc_code(qc_random_shifts(3, 6, 8, seed=1, girth_min=6), 8, "tiny-qc48")


_PEG_CACHE: dict = {}


def peg1008_code(seed: int = 2) -> Code:
    """(3,6)-regular PEG code, N=1008, M=504, redrawn from seed, seed+1000, ...
    until it has no 4-cycle (two checks sharing two variables)."""
    if seed in _PEG_CACHE:
        return _PEG_CACHE[seed]
    s = seed
    while True:
        c = peg_regular(1008, 504, 3, 6, s)
        if _csr_no_4cycle(c):
            break
        s += 1000
    _PEG_CACHE[seed] = c
    return c


def _csr_no_4cycle(c: Code) -> bool:
    pairs = set()
    for r in range(c.m):
        vs = c.col[c.row_ptr[r]:c.row_ptr[r + 1]]
        for a in range(len(vs)):
            for b in range(a + 1, len(vs)):
                key = (int(vs[a]), int(vs[b]))
                if key in pairs:
                    return False
                pairs.add(key)
    return True


def qc2640_code() -> Code:
    """3x6 base, Z=440 (N=2640, M=1320), seed 3, girth >= 8."""
    return qc_code(qc_random_shifts(3, 6, 440, seed=3, girth_min=8), 440, "qc2640")


def table5_code1() -> Code:
    """Code 1 of Section III: the 4x20, L=128 exponent matrix of Table V."""
    path = os.path.join(_GOLDEN, "table5_code1.txt")
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line.startswith("E "):
                rows.append([int(t) for t in line[2:].split()])
    return qc_code(np.array(rows, dtype=np.int32), 128, "table5-code1")


def batch_codes(count: int = 64, seed: int = 4) -> List[Code]:
    """Uneven QC codes: base in {3x6, 4x8, 3x12, 4x24} (all blocks nonzero),
    Z uniform in 16..384, shifts by the greedy 4-cycle-free assignment."""
    rng = np.random.default_rng(seed)
    bases = [(3, 6), (4, 8), (3, 12), (4, 24)]
    out = []
    for idx in range(count):
        mb, nb = bases[int(rng.integers(0, len(bases)))]
        while True:
            z = int(rng.integers(16, 385))
            s = qc_greedy_shifts(np.ones((mb, nb), dtype=bool), z, rng)
            if s is not None:
                break
        out.append(qc_code(s, z, f"batch{idx}-{mb}x{nb}-z{z}"))
    return out


def serving_pool(count: int = 32, seed: int = 5) -> List[Code]:
    """46x68 base with column weights uniform in {3,4,5}, Z uniform in 32..384,
    greedy 4-cycle-free shifts."""
    rng = np.random.default_rng(seed)
    out = []
    for idx in range(count):
        while True:
            mask = np.zeros((46, 68), dtype=bool)
            for j in range(68):
                w = int(rng.integers(3, 6))
                mask[rng.choice(46, size=w, replace=False), j] = True
            if mask.sum(axis=1).min() >= 2:
                break
        while True:
            z = int(rng.integers(32, 385))
            s = qc_greedy_shifts(mask, z, rng)
            if s is not None:
                break
        out.append(qc_code(s, z, f"serve{idx}-z{z}"))
    return out
