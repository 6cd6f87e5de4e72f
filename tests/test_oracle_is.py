"""Oracle pins for the noise source and the importance-sampling estimator.

* Philox4x32-10 (Salmon et al., SC'11) against rocRAND's independent
  open-source implementation, compiled here as a host program;
* Box-Muller normals: moments and tail frequency;
* the mean-shift IS estimator against the closed form Q(sqrt(a)/sigma) of a
  linear test decoder (fails iff the sum of the received TS bits is negative),
  and against plain Monte Carlo when the shift is 0.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

PROBE = r"""
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>
// ten_rounds is a protected member: expose it through a derived class
struct exposed : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
    exposed eng;
    for (int i = 1; i + 5 < argc + 1; i += 6) {
        uint4 c = {(unsigned)strtoul(argv[i], 0, 10), (unsigned)strtoul(argv[i+1], 0, 10),
                   (unsigned)strtoul(argv[i+2], 0, 10), (unsigned)strtoul(argv[i+3], 0, 10)};
        uint2 k = {(unsigned)strtoul(argv[i+4], 0, 10), (unsigned)strtoul(argv[i+5], 0, 10)};
        uint4 r = eng.run(c, k);
        printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


def _probe(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(oracle_mod, tmp_path):
    exe = _probe(tmp_path)
    rng = np.random.default_rng(5)
    cases = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [1, 2, 3, 4, 5, 6]]
    cases += rng.integers(0, 2**32, size=(20, 6), dtype=np.uint64).tolist()
    args = [str(int(x)) for c in cases for x in c]
    out = subprocess.run([str(exe)] + args, check=True, capture_output=True, text=True).stdout
    got = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(got) == len(cases)
    for c, g in zip(cases, got):
        mine = oracle_mod.philox(c[:4], c[4:])
        assert list(map(int, mine)) == g, c


def test_normals_moments(oracle_mod):
    x = np.concatenate([oracle_mod.normals(1234, f, 7, 1000) for f in range(200)])
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0) < 0.01
    assert abs((x > 2.0).mean() - 0.02275) < 0.002
    # distinct frames and streams give distinct draws; the same counter repeats
    assert not np.allclose(oracle_mod.normals(1, 0, 0, 8), oracle_mod.normals(1, 1, 0, 8))
    assert not np.allclose(oracle_mod.normals(1, 0, 0, 8), oracle_mod.normals(1, 0, 1, 8))
    assert np.array_equal(oracle_mod.normals(9, 3, 2, 13), oracle_mod.normals(9, 3, 2, 16)[:13])


def _q(x):
    return 0.5 * math.erfc(x / math.sqrt(2.0))


@pytest.mark.parametrize("ebn0,shift", [(3.0, 1.0), (5.0, 1.0), (4.0, 0.8)])
def test_is_closed_form_linear_decoder(oracle_mod, tiny, ebn0, shift):
    c, oc = tiny
    T = [3, 17, 40, 81]
    a = len(T)
    s2 = oracle_mod.sigma2(ebn0, 0.5)
    exact = _q(math.sqrt(a) / math.sqrt(s2))
    r = oracle_mod.is_estimate(oc, T, ebn0, shift, 40000, seed=99,
                               decoder=oracle_mod.IS_LINEAR)
    sd = math.sqrt(r["var"])
    assert abs(r["p_hat"] - exact) < 3.0 * sd, (r["p_hat"], exact, sd)
    assert abs(r["p_hat"] - exact) / exact < 0.05


def test_is_zero_shift_is_plain_monte_carlo(oracle_mod, tiny):
    c, oc = tiny
    r = oracle_mod.is_estimate(oc, [1, 2], 1.0, 0.0, 5000, seed=3,
                               decoder=oracle_mod.IS_LINEAR, want_fail=True)
    assert r["p_hat"] == r["n_fail"] / 5000 == (r["fail"] & 1).mean()
    assert r["sum_w2"] == r["sum_w"]


def test_is_spa_frames_resumable(oracle_mod, tiny):
    """Counter-based noise: frames [0,N) equal frames [0,N/2) + [N/2,N)."""
    c, oc = tiny
    T = [0, 8, 19]
    full = oracle_mod.is_estimate(oc, T, 3.0, 1.2, 400, seed=5, want_fail=True)
    a = oracle_mod.is_estimate(oc, T, 3.0, 1.2, 200, seed=5, want_fail=True)
    b = oracle_mod.is_estimate(oc, T, 3.0, 1.2, 200, seed=5, frame_base=200, want_fail=True)
    assert np.array_equal(full["fail"], np.concatenate([a["fail"], b["fail"]]))
    assert abs(full["sum_w"] - (a["sum_w"] + b["sum_w"])) <= 1e-12 * max(1.0, full["sum_w"])


@pytest.mark.parametrize("ebn0,shift", [(3.0, 0.5), (4.0, 0.75)])
def test_is_spa_unbiased_against_plain_monte_carlo(oracle_mod, tiny, ebn0, shift):
    """With the real sum-product decoder, the mean-shift estimate (the likelihood
    ratio weights every failure, wherever it comes from) equals plain Monte
    Carlo within the two estimators' combined 3 sigma.  At these SNRs direct
    simulation of the tiny code sees well over 100 failures (about 4200 and
    1000 of 6e4 frames); the two runs use independent Philox streams."""
    c, oc = tiny
    T = [s for a, b, s in oracle_mod.brute_ts_list(oc, 3) if a == 3][0]
    K = 60000
    mc = oracle_mod.is_estimate(oc, T, ebn0, 0.0, K, seed=21, stream=1)
    r = oracle_mod.is_estimate(oc, T, ebn0, shift, K, seed=21, stream=2)
    assert mc["n_fail"] >= 100 and r["n_fail"] >= 100
    z = (r["p_hat"] - mc["p_hat"]) / math.sqrt(r["var"] + mc["var"])
    print(f"\nIS SPA {ebn0} dB s={shift}: plain MC {mc['p_hat']:.4e} ({mc['n_fail']} failures), "
          f"IS {r['p_hat']:.4e} (rel. sd {math.sqrt(r['var']) / r['p_hat']:.3f}), z = {z:.2f}")
    assert abs(z) < 3.0


def test_is_count_ts_events(oracle_mod, tiny):
    """Counting only the set's own error events (every bit of T and at most 2a
    bits in error at the end): flag bit 1 implies bit 0, it matches a re-decode
    of the frame, and the estimate is the sum over exactly those frames."""
    c, oc = tiny
    T = [s for a, b, s in oracle_mod.brute_ts_list(oc, 3) if a == 3][0]
    ebn0, shift, K = 3.0, 1.5, 3000
    al = oracle_mod.is_estimate(oc, T, ebn0, shift, K, seed=4, stream=9, want_fail=True)
    ts = oracle_mod.is_estimate(oc, T, ebn0, shift, K, seed=4, stream=9, want_fail=True,
                                count_mode=oracle_mod.IS_COUNT_TS)
    assert np.array_equal(al["fail"], ts["fail"])
    f = ts["fail"]
    assert ((f & 2) == 0).all() or (f[(f & 2) != 0] & 1).all()
    assert ts["n_fail"] == int(((f >> 1) & 1).sum()) and al["n_fail"] == int((f & 1).sum())
    assert 0 < ts["n_fail"] < al["n_fail"]
    assert ts["p_hat"] <= al["p_hat"]
    s2 = oracle_mod.sigma2(ebn0, 0.5)
    sig = math.sqrt(s2)
    rng = np.random.default_rng(2)
    for fr in rng.choice(K, 40, replace=False):
        n = oracle_mod.normals(4, int(fr), 9, oc.n)
        y = 1.0 + sig * n
        y[list(T)] -= shift
        d = oracle_mod.decode_spa(oc, 2.0 * y / s2, 50)
        err = d["app"] < 0
        want = d["fail"] and err[list(T)].all() and err.sum() <= 2 * len(T)
        assert bool(f[fr] & 1) == bool(d["fail"]) and bool(f[fr] & 2) == bool(want), fr


def test_is_pilot_shift_rule(oracle_mod, tiny):
    """The pilot rule picks, among the grid eps* (1/2 + i/16), the point with
    the smallest relative variance (at least 10 counted failures), each point
    estimated on its own frames frame_base + 2^40 + i P."""
    c, oc = tiny
    T = [s for a, b, s in oracle_mod.brute_ts_list(oc, 3) if a == 3][0]
    ebn0, P = 4.0, 600
    eps = oracle_mod.spa_eps_star(oc, T, ebn0)
    s, rv = oracle_mod.is_pilot_shift(oc, T, ebn0, eps, P, seed=3, stream=5,
                                      count_mode=oracle_mod.IS_COUNT_TS)
    want = []
    for i in range(9):
        r = oracle_mod.is_estimate(oc, T, ebn0, eps * (0.5 + i / 16.0), P, seed=3, stream=5,
                                   frame_base=(1 << 40) + i * P, count_mode=oracle_mod.IS_COUNT_TS)
        want.append(r["var"] / r["p_hat"] ** 2 if r["n_fail"] >= 10 else -1.0)
    assert np.allclose(rv, want, rtol=1e-12)
    ok = [i for i in range(9) if want[i] >= 0]
    assert ok
    best = min(ok, key=lambda i: (want[i], i))
    assert s == eps * (0.5 + best / 16.0)


@pytest.mark.parametrize("ebn0,s0,ds,m", [(3.0, 0.5, 0.125, 9), (5.0, 0.6, 0.1, 5)])
def test_is_mixture_closed_form_linear_decoder(oracle_mod, tiny, ebn0, s0, ds, m):
    """Mixture of shifts (balance heuristic) against the exact Q(sqrt(a)/sigma)
    of the linear test decoder: within 3 sigma and 5%."""
    c, oc = tiny
    T = [3, 17, 40, 81]
    a = len(T)
    s2 = oracle_mod.sigma2(ebn0, 0.5)
    exact = _q(math.sqrt(a) / math.sqrt(s2))
    r = oracle_mod.is_estimate(oc, T, ebn0, 0.0, 45000, seed=98, decoder=oracle_mod.IS_LINEAR,
                               mix=(m, s0, ds))
    sd = math.sqrt(r["var"])
    assert abs(r["p_hat"] - exact) < 3.0 * sd, (r["p_hat"], exact, sd)
    assert abs(r["p_hat"] - exact) / exact < 0.05
    assert r["shift_used"] == pytest.approx(s0 + (m - 1) * ds)


def test_is_mixture_of_one_is_the_single_shift(oracle_mod, tiny):
    c, oc = tiny
    T = [0, 8, 19]
    one = oracle_mod.is_estimate(oc, T, 3.0, 1.3, 600, seed=5, want_fail=True)
    mix = oracle_mod.is_estimate(oc, T, 3.0, 0.0, 600, seed=5, want_fail=True, mix=(1, 1.3, 0.0))
    assert np.array_equal(one["fail"], mix["fail"])
    assert mix["p_hat"] == pytest.approx(one["p_hat"], rel=1e-12)
    assert mix["var"] == pytest.approx(one["var"], rel=1e-9)
