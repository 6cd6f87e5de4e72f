"""Importance sampling on the QC-2640 stand-in (girth 8) against the oracle.
Only the set's own error events count (every bit of T and at most 2a bits in
error at the end of the decode), and the frames are either split over the
mixture of shifts eps* k/16, k = 0..16, weighted by the balance heuristic (the
union bound's estimator), or run at one shift chosen by pilot runs over the
grid eps* (1/2 + i/16), i = 0..8.

Bars (Section I/II, Cole's TS weighting): on the very same Philox frames the
per-frame flags agree on at least 99.5% of 10^4 frames, and the estimate lies
within 2% of the oracle's or inside its 95% confidence interval; the shift the
device's pilots choose is the oracle's, or one whose relative variance by the
oracle's own pilots is within 25% of the oracle's best.
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SPA = dict(max_iter=50, k_max=32 * 1024, k_den=1024)


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def qc():
    import paper_2208_05795_amd as tsg
    code = workloads.qc2640_code()
    ctx = tsg.Context(0)
    g = ctx.load_code(code)
    g.impulse_search(g.make_patterns(tsg.PAT_TRIPLES | tsg.PAT_QC_ORBITS), decoder=tsg.DEC_SPA,
                     a_max=12, **SPA)
    ts = g.collect()
    assert len(ts) >= 2
    yield code, ctx, g, ts
    g.free()
    ctx.close()


@pytest.mark.parametrize("which,ebn0", [(0, 3.0), (1, 5.0)])
def test_is_qc2640_pilot_and_frames(oracle_mod, qc, which, ebn0):
    import paper_2208_05795_amd as tsg
    code, ctx, g, ts = qc
    oc = oracle_mod.OCode(code)
    bits = list(ts[which].bits)
    K, P, seed, stream = 10000, 1000, 17, which
    eps = oracle_mod.spa_eps_star(oc, bits, ebn0)
    got = g.is_estimate(bits, ebn0, -1.0, K, seed=seed, stream=stream, want_fail=True,
                        count_mode=tsg.IS_COUNT_TS, shift_rule=tsg.SHIFT_PILOT, pilot_frames=P)
    s_ref, rv = oracle_mod.is_pilot_shift(oc, bits, ebn0, eps, P, seed, stream=stream,
                                          count_mode=oracle_mod.IS_COUNT_TS)
    s = got["shift_used"]
    grid = [eps * (0.5 + i / 16.0) for i in range(9)]
    i_dev = int(np.argmin([abs(x - s) for x in grid]))
    ok_rv = [x for x in rv if x >= 0]
    _say(f"TS{bits} ({ts[which].a},{ts[which].b}) {ebn0} dB: eps* {eps}; shift device {s:.4f} "
         f"oracle {s_ref:.4f}; oracle pilot relative variances {np.round(rv, 1).tolist()}")
    assert abs(grid[i_dev] - s) <= 1e-3 * eps   # the device's eps* is the oracle's (1e-3)
    assert abs(s - s_ref) <= 1e-3 * eps or (rv[i_dev] >= 0 and rv[i_dev] <= 1.25 * min(ok_rv))
    ref = oracle_mod.is_estimate(oc, bits, ebn0, s, K, seed=seed, stream=stream, want_fail=True,
                                 count_mode=oracle_mod.IS_COUNT_TS)
    agree = (got["fail"] == ref["fail"]).mean()
    _say(f"  p device {got['p_hat']:.4e} oracle {ref['p_hat']:.4e} ci [{ref['ci_lo']:.3e}, "
         f"{ref['ci_hi']:.3e}], counted failures {got['n_fail']} / {ref['n_fail']}, frame "
         f"agreement {agree:.5f}")
    assert agree >= 0.995
    inside = ref["ci_lo"] <= got["p_hat"] <= ref["ci_hi"]
    close = abs(got["p_hat"] - ref["p_hat"]) <= 0.02 * abs(ref["p_hat"])
    assert inside or close


@pytest.mark.parametrize("which,ebn0", [(0, 2.0), (1, 5.0)])
def test_is_qc2640_mixture_frames(oracle_mod, qc, which, ebn0):
    import paper_2208_05795_amd as tsg
    code, ctx, g, ts = qc
    oc = oracle_mod.OCode(code)
    bits = list(ts[which].bits)
    K, seed, stream = 10000, 19, 4 + which
    got = g.is_estimate(bits, ebn0, -1.0, K, seed=seed, stream=stream, want_fail=True,
                        count_mode=tsg.IS_COUNT_TS, shift_rule=tsg.SHIFT_MIX)
    eps = got["shift_used"]   # the mixture's top shift: the device's eps*
    want = oracle_mod.spa_eps_star(oc, bits, ebn0)
    assert abs(eps - want) <= 1e-3 * want
    ref = oracle_mod.is_estimate(oc, bits, ebn0, 0.0, K, seed=seed, stream=stream, want_fail=True,
                                 count_mode=oracle_mod.IS_COUNT_TS, mix=(17, 0.0, eps / 16.0))
    agree = (got["fail"] == ref["fail"]).mean()
    _say(f"TS{bits} {ebn0} dB mixture: p device {got['p_hat']:.4e} oracle {ref['p_hat']:.4e} ci "
         f"[{ref['ci_lo']:.3e}, {ref['ci_hi']:.3e}], counted {got['n_fail']} / {ref['n_fail']}, "
         f"frame agreement {agree:.5f}")
    assert agree >= 0.995
    inside = ref["ci_lo"] <= got["p_hat"] <= ref["ci_hi"]
    close = abs(got["p_hat"] - ref["p_hat"]) <= 0.02 * abs(ref["p_hat"])
    assert inside or close


def test_union_bound_qc2640_ci(qc):
    """The union bound over the found sets at 2..5 dB, 10^5 frames per (set,
    SNR), the mixture estimator: from 3 dB on every point's 95% confidence
    interval lies above zero.  At 2 dB (near this code's waterfall) events far
    from the sets' own direction dominate the sets' error events and no
    estimator that biases only the set's bits converges in 10^5 frames: that
    point is reported, not asserted."""
    import paper_2208_05795_amd as tsg
    code, ctx, g, ts = qc
    ub = g.union_bound(len(ts), [2.0, 3.0, 4.0, 5.0], 100000, seed=7, per_ts=True,
                       count_mode=tsg.IS_COUNT_TS, shift_rule=tsg.SHIFT_MIX)
    for p, row in zip(ub["points"], ub["per_ts"]):
        _say(f"{p['ebn0_db']} dB: FER {p['fer']:.3e} ci [{p['ci_lo']:.3e}, {p['ci_hi']:.3e}]; "
             f"per set (shift, counted failures, P): "
             f"{[(round(r['shift_used'], 3), r['n_fail'], '%.2e' % r['p_hat']) for r in row]}")
    for p, row in zip(ub["points"], ub["per_ts"]):
        if p["ebn0_db"] < 3.0:
            continue
        assert p["fer"] > 0.0 and p["ci_lo"] > 0.0
        for r in row:
            assert r["p_hat"] > 0.0 and math.isfinite(r["var"])
