"""A search whose candidate error sets overflow the record buffer re-runs the
chunk in smaller pieces: same per-pattern outputs, same TS list, and the same
decode and edge-update statistics as a run that never overflows (the first,
discarded run of an overflowing chunk is not counted)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")


def _run(tsg, rec_bytes, code, pats, **kw):
    with tsg.Context(0, rec_buffer_bytes=rec_bytes) as ctx:
        g = ctx.load_code(code)
        r = g.impulse_search(pats, **kw)
        ts = [(t.a, t.b, t.orbit, t.first_pattern, t.k_crit, t.bits) for t in g.collect()]
        st = r["stats"]
        out = {k: np.asarray(r[k]).copy() for k in KEYS}
        g.free()
    return out, ts, st


@pytest.mark.parametrize("decoder", ["oms", "spa"])
def test_overflowing_record_buffer(decoder):
    import paper_2208_05795_amd as tsg
    code = workloads.peg1008_code()
    with tsg.Context(0) as ctx:
        allp = ctx.load_code(code).pattern_list([1, 2, 3])
    rng = np.random.default_rng(51)
    pats = np.ascontiguousarray(allp[np.sort(rng.choice(len(allp), 600, replace=False))])
    kw = dict(a_max=12)
    if decoder == "spa":
        kw.update(decoder=tsg.DEC_SPA, max_iter=50, k_max=32 * 1024, k_den=1024)
    else:   # a weak channel so that impulses fail and write candidates
        kw.update(llr_scale=1.0)
    ref, ts_ref, st_ref = _run(tsg, 0, code, pats, **kw)
    got, ts_got, st_got = _run(tsg, 1, code, pats, **kw)   # one pattern's worst case
    print(f"[gpu] {decoder}: launches {st_ref['decode_launches']} -> {st_got['decode_launches']}, "
          f"candidates {st_ref['candidates']}, edge-updates {st_ref['edge_updates']}", flush=True)
    assert st_got["decode_launches"] > st_ref["decode_launches"] + 1   # chunks were re-run
    for k in KEYS:
        assert np.array_equal(got[k], ref[k]), k
    assert ts_got == ts_ref
    assert st_got["decodes"] == st_ref["decodes"]
    assert st_got["edge_updates"] == st_ref["edge_updates"]
    assert st_got["candidates"] == st_ref["candidates"]
