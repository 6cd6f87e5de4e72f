"""ts_is_estimate_noalloc (the IS estimate with every device buffer in the
library's fixed device array) against ts_is_estimate, through the C ABI: two
calls in a row, the second with fewer frames, each identical to the allocating
call on the same frames (estimate, sums, counted failures, per-frame flags);
and the limits are refused with an error."""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _call(tsg, A, fn, g, bits, frames, **kw):
    t = np.ascontiguousarray(np.asarray(bits, dtype=np.int32))
    o = A.IsOpts(kw.get("max_iter", 50), kw["ebn0_db"], 1.0 - g.m / g.n, kw["shift"], frames,
                 kw["seed"], kw.get("frame_base", 0), kw.get("stream", 0), 0, 0,
                 kw.get("count_mode", 0), 0, 0)
    r = A.IsResult()
    fl = np.zeros(frames, dtype=np.uint8)
    rc = fn(g.ctx.handle, g._h, t.ctypes.data, t.size, C.byref(o), C.byref(r), fl.ctypes.data)
    if rc != A.TS_OK:
        raise tsg.TsgError(rc, tsg.lib().ts_last_error().decode())
    out = {f: getattr(r, f) for f, _ in A.IsResult._fields_}
    out["fail"] = fl
    out["stats"] = g.ctx.stats()
    return out


@pytest.mark.parametrize("name", ["tiny", "peg1008"])
def test_noalloc_matches_allocating_call(name):
    import paper_2208_05795_amd as tsg
    from paper_2208_05795_amd import _capi as A
    L = tsg.lib()
    code = workloads.tiny_code() if name == "tiny" else workloads.peg1008_code()
    with tsg.Context(0) as ctx:
        g = ctx.load_code(code)
        rp, col = g.csr()
        bits = sorted(set(int(x) for x in col[rp[0]:rp[1]]))[:4]
        sh = 1.2 if name == "tiny" else 2.5   # shifts at which frames fail
        counted = 0
        for frames, ebn0, cm in ((20000, 3.0, 0), (3000, 2.5, 0)):
            kw = dict(ebn0_db=ebn0, shift=sh, seed=31, stream=2, count_mode=cm)
            ref = _call(tsg, A, L.ts_is_estimate, g, bits, frames, **kw)
            got = _call(tsg, A, L.ts_is_estimate_noalloc, g, bits, frames, **kw)
            _say(f"{name} {frames} frames {ebn0} dB: p {got['p_hat']:.4e} vs {ref['p_hat']:.4e}, "
                 f"counted {got['n_fail']}, edge-updates {got['stats']['edge_updates']} vs "
                 f"{ref['stats']['edge_updates']}")
            assert np.array_equal(got["fail"], ref["fail"])
            for k in ("p_hat", "var", "ci_lo", "ci_hi", "sum_w", "sum_w2", "n", "n_fail", "shift_used"):
                assert got[k] == ref[k], k
            assert got["n"] == frames
            assert got["stats"]["edge_updates"] == ref["stats"]["edge_updates"]
            counted += got["n_fail"]
        assert counted > 0
        g.free()


def test_noalloc_limits():
    import paper_2208_05795_amd as tsg
    from paper_2208_05795_amd import _capi as A
    L = tsg.lib()
    with tsg.Context(0) as ctx:
        g = ctx.load_code(workloads.tiny_code())
        with pytest.raises(tsg.TsgError):   # no eps* search without allocating
            _call(tsg, A, L.ts_is_estimate_noalloc, g, [0, 1], 100, ebn0_db=3.0, shift=-1.0, seed=1)
        with pytest.raises(tsg.TsgError):   # beyond the array
            _call(tsg, A, L.ts_is_estimate_noalloc, g, [0, 1], (1 << 21) + 1, ebn0_db=3.0,
                  shift=1.0, seed=1)
        g.free()
