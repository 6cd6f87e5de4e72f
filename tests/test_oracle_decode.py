"""Oracle pins: decoder arithmetic and channel values.

OMS: hand-computed first iterations on the tiny code.  SPA: on a cycle-free
Tanner graph flooding sum-product converges to the exact bitwise MAP posterior,
computed here by brute-force marginalisation over all codewords.
"""
import itertools
import math

import numpy as np
import pytest

import workloads


def test_channel_values(oracle_mod):
    # sigma^2 = 1/(2 R 10^(EbN0/10)); h = 2/sigma^2 at 3 dB, R = 1/2 is 3.99052
    s2 = oracle_mod.sigma2(3.0, 0.5)
    assert abs(2.0 / s2 - 3.990524) < 1e-5
    assert oracle_mod.q_base(3.0, 0.5) == 16          # round(4 h)
    assert oracle_mod.q_base(5.0, 0.5) == 25          # 4 * 6.32456 = 25.3
    qb = 16
    # lambda = h (1 - k/16) on the int8 scale: 16 - k until saturation at -127
    for k in range(0, 200):
        assert oracle_mod.q_impulse(qb, k) == max(16 - k, -127)
    # rounding half away from zero: q_base 9, k = 8 -> 4.5 -> 5; k = 24 -> -4.5 -> -5
    assert oracle_mod.q_impulse(9, 8) == 5 and oracle_mod.q_impulse(9, 24) == -5
    assert oracle_mod.q_impulse(127, 512) == -127


def test_oms_noiseless_first_iteration(oracle_mod, tiny):
    c, oc = tiny
    r = oracle_mod.decode_oms(oc, np.full(oc.n, 16), 20, 1)
    # every check sends min(16) - 1 = 15 to every variable: APP = 16 + 3*15
    assert (r["fail"], r["iters"], r["tmin"]) == (0, 1, 1)
    assert (r["app"] == 61).all()


@pytest.mark.parametrize("k", [8, 16, 17, 40, 512])
def test_oms_single_impulse_first_iteration(oracle_mod, tiny, k):
    c, oc = tiny
    qb = 16
    qi = oracle_mod.q_impulse(qb, k)
    q = np.full(oc.n, qb)
    v0 = 5
    q[v0] = qi
    r = oracle_mod.decode_oms(oc, q, 1, 1)
    app = r["app"]
    rp, col = oc.csr()
    nbrs = set()
    for row in range(oc.m):
        vs = col[rp[row]:rp[row + 1]]
        if v0 in vs:
            nbrs.update(int(v) for v in vs if v != v0)
    sgn = 1 if qi >= 0 else -1
    to_nbr = sgn * max(min(abs(qi), qb) - 1, 0)
    assert app[v0] == qi + 3 * 15
    for v in range(oc.n):
        if v in nbrs:
            assert app[v] == qb + 2 * 15 + to_nbr
        elif v != v0:
            assert app[v] == qb + 45


def test_oms_offset_and_saturation(oracle_mod):
    """One check of degree 3 with channel values (100, -3, 0): messages use
    v2c saturated to [-127, 127], sgn(0) = +1 and max(min - beta, 0)."""
    oc = oracle_mod.OCode(workloads.csr_code(3, 1, [0, 3], [0, 1, 2]))
    r = oracle_mod.decode_oms(oc, [100, -3, 0], 1, 1)
    # to v0: sgn(-3)*sgn(0) * max(min(3,0)-1,0) = 0 ; to v1: + * max(0-1,0) = 0
    # to v2: sgn(100)*sgn(-3) * max(3-1, 0) = -2
    assert list(r["app"]) == [100, -3, -2]
    r = oracle_mod.decode_oms(oc, [127, 127, -127], 1, 2)
    # to v0: - * (127-2) = -125; v1 likewise; to v2: + (127 - 2)
    assert list(r["app"]) == [2, 2, -2]


def _map_llr(H, lam):
    """Exact bitwise MAP LLRs by marginalising over all codewords of H."""
    m, n = H.shape
    num = np.zeros(n)
    den = np.zeros(n)
    for bits in itertools.product([0, 1], repeat=n):
        x = np.array(bits)
        if ((H @ x) % 2).any():
            continue
        w = math.exp(-float(np.dot(lam, x)))
        num += w * (x == 0)
        den += w * (x == 1)
    return np.log(num / den)


def test_spa_exact_map_on_cycle_free_graph(oracle_mod):
    rows = [[0, 1, 2], [2, 3, 4], [4, 5], [1, 6], [6, 7, 8]]
    n = 9
    rp = np.cumsum([0] + [len(r) for r in rows])
    oc = oracle_mod.OCode(workloads.csr_code(n, len(rows), rp, np.concatenate(rows)))
    assert oc.girth == 0
    H = np.zeros((len(rows), n), dtype=np.int64)
    for i, r in enumerate(rows):
        H[i, r] = 1
    rng = np.random.default_rng(11)
    for _ in range(5):
        lam = rng.uniform(0.2, 3.0, n) * rng.choice([-1, 1], n)
        r = oracle_mod.decode_spa(oc, lam, max_iter=12, early_stop=False)
        assert np.allclose(r["app"], _map_llr(H, lam), atol=1e-9, rtol=0)


def test_spa_noiseless_decodes_at_once(oracle_mod, tiny):
    c, oc = tiny
    h = 2.0 / oracle_mod.sigma2(3.0, 0.5)
    r = oracle_mod.decode_spa(oc, np.full(oc.n, h), 50)
    assert (r["fail"], r["iters"]) == (0, 1)


def test_decode_stops_on_nonzero_codeword_is_failure(oracle_mod, tiny, tiny_search):
    """The (4,0) set found by the search is a codeword: a channel pointing at it
    converges to it with syndrome 0 and counts as a failure (Section II: TS(a,0)
    are codewords)."""
    c, oc = tiny
    _, res = tiny_search
    cw = [r for r in res["ts"] if r.b == 0][0].bits
    q = np.full(oc.n, 16)
    q[list(cw)] = -40
    r = oracle_mod.decode_oms(oc, q, 20, 1, hist=True)
    assert r["fail"] == 1 and r["synd"][-1] == 0
    assert set(np.nonzero(r["hist"][-1])[0]) == set(cw)


# ---- quantised normalised layered min-sum (4/4/6 bits) -----------------------

def test_lnms_noiseless_tiny_by_hand(oracle_mod, tiny):
    """Every variable of the tiny 3x6 code lies in one check of each block row
    (layer).  With channel value 4 everywhere: layer 0 sends floor(3*4/4) = 3
    (APP 7), layer 1 floor(3*7/4) = 5 (APP 12), layer 2 sat7(floor(3*12/4) = 9)
    = 7 (APP 19); the syndrome is 0 after the first iteration."""
    c, oc = tiny
    n_layers, lay = oracle_mod.layers(oc)
    assert n_layers == 3 and list(lay) == [r // c.z for r in range(c.m)]
    r = oracle_mod.decode_lnms(oc, np.full(oc.n, 4), max_iter=20)
    assert r["iters"] == 1 and r["fail"] == 0
    assert (r["app"] == 19).all()


def test_lnms_two_layers_by_hand(oracle_mod):
    """Checks {0,1,2} and {2,3,4} share variable 2, so they form two layers.
    Channel (4, 4, -3, 4, 4): layer 0 sends -floor(3*3/4) = -2 to variables 0
    and 1 (APP 2, 2) and +floor(3*4/4) = 3 to variable 2 (APP 0); layer 1 reads
    v2c 0 from variable 2, sends it +3 (APP 3) and, through the zero (sign +),
    +0 to variables 3 and 4 (APP 4, 4).  Channel (7, 7, -7, 7, 7): layer 0 gives
    APP (2, 2, -2); layer 1 sends +5 to variable 2 (APP 3) and -floor(3*2/4) =
    -1 to variables 3 and 4 (APP 6, 6)."""
    oc = oracle_mod.OCode(workloads.csr_code(5, 2, [0, 3, 6], [0, 1, 2, 2, 3, 4]))
    n_layers, lay = oracle_mod.layers(oc)
    assert n_layers == 2 and list(lay) == [0, 1]
    r = oracle_mod.decode_lnms(oc, [4, 4, -3, 4, 4], max_iter=1)
    assert list(r["app"]) == [2, 2, 3, 4, 4] and r["iters"] == 1 and r["fail"] == 0
    r = oracle_mod.decode_lnms(oc, [7, 7, -7, 7, 7], max_iter=1)
    assert list(r["app"]) == [2, 2, 3, 6, 6]
    # channel values are 4-bit: out-of-range inputs saturate on entry
    r = oracle_mod.decode_lnms(oc, [100, 100, -100, 100, 100], max_iter=1)
    assert list(r["app"]) == [2, 2, 3, 6, 6]


def test_lnms_layers_and_ranges(oracle_mod):
    """Greedy layers of a CSR code: each layer's checks touch disjoint
    variables, and every check sits in the lowest layer free of its variables
    at its turn.  APP values stay within 6 bits."""
    code = workloads.peg1008_code()
    oc = oracle_mod.OCode(code)
    n_layers, lay = oracle_mod.layers(oc)
    rp, col = oc.csr()
    owner = {}
    for r in range(oc.m):
        vs = col[rp[r]:rp[r + 1]]
        free = next(L for L in range(n_layers + 1) if all((int(v), L) not in owner for v in vs))
        assert lay[r] == free
        for v in vs:
            owner[(int(v), int(lay[r]))] = r
    assert n_layers == max(lay) + 1
    rng = np.random.default_rng(5)
    q = rng.integers(-7, 8, size=oc.n)
    r = oracle_mod.decode_lnms(oc, q, max_iter=20)
    assert np.abs(r["app"]).max() <= 31


def test_lnms_channel_values(oracle_mod):
    qb = oracle_mod.q4_base(3.0, 0.5, 1.0)
    assert qb == 4   # round(3.99)
    assert [oracle_mod.q4_impulse(qb, k) for k in (0, 4, 8, 16, 32, 64, 512)] == [4, 3, 2, 0, -4, -7, -7]
    assert oracle_mod.q4_base(3.0, 0.5, 4.0) == 7   # saturated
