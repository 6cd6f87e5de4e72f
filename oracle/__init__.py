"""Python access to the CPU oracle (test infrastructure only).

The oracle is the plain C reference in this directory (see oracle.h).  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg import it; the
GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PAT_SINGLES, PAT_PAIRS, PAT_TRIPLES = 1, 2, 3
DEC_OMS, DEC_SPA, DEC_LNMS = 0, 1, 2
EXTRACT_PATH, EXTRACT_CRITICAL = 0, 1

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class DecResult(C.Structure):
    _fields_ = [("fail", C.c_int32), ("iters", C.c_int32), ("tmin", C.c_int32),
                ("wmin", C.c_int32)]


class SearchOpts(C.Structure):
    _fields_ = [("decoder", C.c_int32), ("max_iter", C.c_int32), ("oms_offset", C.c_int32),
                ("ebn0_db", C.c_double), ("rate", C.c_double), ("llr_scale", C.c_double),
                ("k_max", C.c_int32), ("k_den", C.c_int32), ("a_max", C.c_int32),
                ("extract_mode", C.c_int32), ("collect_from_iter", C.c_int32),
                ("threads", C.c_int32), ("spa_grid", C.c_int32)]


class IsOpts(C.Structure):
    _fields_ = [("decoder", C.c_int32), ("max_iter", C.c_int32), ("ebn0_db", C.c_double), ("rate", C.c_double),
                ("shift", C.c_double), ("n_frames", C.c_int64), ("seed", C.c_uint64),
                ("frame_base", C.c_uint64), ("stream", C.c_uint32), ("threads", C.c_int32),
                ("count_mode", C.c_int32), ("n_mix", C.c_int32), ("mix_s0", C.c_double),
                ("mix_ds", C.c_double)]


class IsResult(C.Structure):
    _fields_ = [("p_hat", C.c_double), ("var", C.c_double), ("ci_lo", C.c_double),
                ("ci_hi", C.c_double), ("sum_w", C.c_double), ("sum_w2", C.c_double),
                ("n", C.c_int64), ("n_fail", C.c_int64), ("shift_used", C.c_double)]


def lib():
    """Loads liboracle.so, building it first when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    L.or_code_qc.restype = vp
    L.or_code_qc.argtypes = [C.c_int, C.c_int, C.c_int, _i32p]
    L.or_code_csr.restype = vp
    L.or_code_csr.argtypes = [C.c_int, C.c_int, _i64p, _i32p]
    L.or_code_free.argtypes = [vp]
    L.or_code_info.argtypes = [vp] + [C.POINTER(C.c_int32)] * 2 + [C.POINTER(C.c_int64)] + \
        [C.POINTER(C.c_int32)] * 2
    L.or_code_csr_out.argtypes = [vp, _i64p, _i32p]
    L.or_sigma2.restype = C.c_double
    L.or_sigma2.argtypes = [C.c_double, C.c_double]
    L.or_q_base.argtypes = [C.c_double, C.c_double, C.c_double]
    L.or_q_impulse.argtypes = [C.c_int, C.c_int]
    L.or_decode_oms.restype = DecResult
    L.or_decode_oms.argtypes = [vp, _i32p, C.c_int, C.c_int, vp, vp]
    L.or_decode_spa.restype = DecResult
    L.or_decode_spa.argtypes = [vp, _f64p, C.c_int, vp, vp, vp]
    L.or_decode_oms_ex.restype = DecResult
    L.or_decode_oms_ex.argtypes = [vp, _i32p, C.c_int, C.c_int, vp, vp, vp]
    L.or_decode_lnms.restype = DecResult
    L.or_decode_lnms.argtypes = [vp, _i32p, C.c_int, vp, vp, vp]
    L.or_layers.argtypes = [vp, _i32p]
    L.or_q4_base.argtypes = [C.c_double, C.c_double, C.c_double]
    L.or_q4_impulse.argtypes = [C.c_int, C.c_int]
    L.or_decode_spa_ex.restype = DecResult
    L.or_decode_spa_ex.argtypes = [vp, _f64p, C.c_int, vp, vp, vp, C.c_int]
    L.or_decode_spa_grid.restype = DecResult
    L.or_decode_spa_grid.argtypes = [vp, _f64p, C.c_int, vp, vp, vp, C.c_int, C.c_int]
    L.or_patterns.restype = C.c_int64
    L.or_patterns.argtypes = [vp, C.c_int, vp, C.c_int64]
    L.or_count_b.argtypes = [vp, _i32p, C.c_int]
    L.or_tree.argtypes = [vp, _i32p, C.c_int, _i32p]
    L.or_ts_closure.argtypes = [vp, _i32p, C.c_int, _i32p]
    L.or_canon.argtypes = [vp, _i32p, C.c_int, _i32p, C.POINTER(C.c_int32)]
    L.or_search.argtypes = [vp, C.POINTER(SearchOpts), _i32p, C.c_int32, C.c_int32] + \
        [_i32p] * 5 + [C.POINTER(C.c_int64)] * 2 + [C.POINTER(vp)]
    L.or_ts_count.restype = C.c_int64
    L.or_ts_count.argtypes = [vp]
    L.or_ts_get.argtypes = [vp, C.c_int64] + [C.POINTER(C.c_int32)] * 5 + [_i32p]
    L.or_ts_free.argtypes = [vp]
    L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.or_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, _f64p]
    L.or_is_estimate.argtypes = [vp, _i32p, C.c_int, C.POINTER(IsOpts), C.POINTER(IsResult),
                                 vp, C.POINTER(C.c_int64)]
    L.or_is_pilot_shift.restype = C.c_double
    L.or_is_pilot_shift.argtypes = [vp, _i32p, C.c_int, C.POINTER(IsOpts), C.c_double, C.c_int64,
                                    _f64p]
    L.or_spa_eps_star.restype = C.c_double
    L.or_spa_eps_star.argtypes = [vp, _i32p, C.c_int, C.c_double, C.c_double, C.c_int,
                                  C.c_double]
    L.or_brute_ts.restype = C.c_int64
    L.or_brute_ts.argtypes = [vp, C.c_int, C.c_int, _i64p, _i64p]
    L.or_brute_ts_list.restype = C.c_int64
    L.or_brute_ts_list.argtypes = [vp, C.c_int, vp, C.c_int64]
    L.or_dmin.argtypes = [vp, _i32p]
    L.or_cycle_emd.argtypes = [vp, C.c_int, C.c_int, _i64p, vp, vp]
    _lib = L
    return L


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class OCode:
    """The oracle's own copy of a code (it expands QC form itself)."""

    def __init__(self, code):
        L = lib()
        if code.kind == "qc":
            h = L.or_code_qc(code.mb, code.nb, code.z, _i32(code.shifts).ravel())
        else:
            h = L.or_code_csr(code.n, code.m, np.ascontiguousarray(code.row_ptr, dtype=np.int64),
                              _i32(code.col))
        if not h:
            raise ValueError("oracle rejected the code")
        self._h = h
        self.code = code
        n, m, g, z = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        e = C.c_int64()
        L.or_code_info(h, C.byref(n), C.byref(m), C.byref(e), C.byref(g), C.byref(z))
        self.n, self.m, self.e, self.girth, self.z = n.value, m.value, e.value, g.value, z.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_code_free(self._h)
            self._h = None

    def csr(self) -> Tuple[np.ndarray, np.ndarray]:
        rp = np.zeros(self.m + 1, dtype=np.int64)
        col = np.zeros(self.e, dtype=np.int32)
        lib().or_code_csr_out(self._h, rp, col)
        return rp, col


def sigma2(ebn0_db: float, rate: float) -> float:
    return lib().or_sigma2(ebn0_db, rate)


def q_base(ebn0_db: float, rate: float, scale: float = 4.0) -> int:
    return lib().or_q_base(ebn0_db, rate, scale)


def q_impulse(qb: int, k: int) -> int:
    return lib().or_q_impulse(qb, k)


def decode_oms(oc: OCode, q_llr, max_iter: int = 20, offset: int = 1, hist: bool = False):
    q = _i32(q_llr)
    hb = np.zeros((max_iter, oc.n), dtype=np.uint8) if hist else None
    sy = np.zeros(max_iter, dtype=np.int32)
    app = np.zeros(oc.n, dtype=np.int32)
    r = lib().or_decode_oms_ex(oc.handle, q, max_iter, offset,
                               hb.ctypes.data if hist else None, sy.ctypes.data, app.ctypes.data)
    out = dict(fail=r.fail, iters=r.iters, tmin=r.tmin, wmin=r.wmin, synd=sy[:r.iters], app=app)
    if hist:
        out["hist"] = hb[:r.iters]
    return out


def decode_lnms(oc: OCode, q_llr, max_iter: int = 20, hist: bool = False):
    """Quantised normalised layered min-sum (4-bit channel / c2v, 6-bit v2c / APP)."""
    q = _i32(q_llr)
    hb = np.zeros((max_iter, oc.n), dtype=np.uint8) if hist else None
    sy = np.zeros(max_iter, dtype=np.int32)
    app = np.zeros(oc.n, dtype=np.int32)
    r = lib().or_decode_lnms(oc.handle, q, max_iter, hb.ctypes.data if hist else None,
                             sy.ctypes.data, app.ctypes.data)
    out = dict(fail=r.fail, iters=r.iters, tmin=r.tmin, wmin=r.wmin, synd=sy[:r.iters], app=app)
    if hist:
        out["hist"] = hb[:r.iters]
    return out


def layers(oc: OCode) -> Tuple[int, np.ndarray]:
    """Layer of every check in the layered schedule, and the number of layers."""
    lay = np.zeros(max(oc.m, 1), dtype=np.int32)
    n = lib().or_layers(oc.handle, lay)
    return n, lay[:oc.m]


def q4_base(ebn0_db: float, rate: float, scale: float = 1.0) -> int:
    return lib().or_q4_base(ebn0_db, rate, scale)


def q4_impulse(qb: int, k: int) -> int:
    return lib().or_q4_impulse(qb, k)


def decode_spa(oc: OCode, llr, max_iter: int = 50, hist: bool = False, early_stop: bool = True,
               grid: int = 0):
    l = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    hb = np.zeros((max_iter, oc.n), dtype=np.uint8) if hist else None
    sy = np.zeros(max_iter, dtype=np.int32)
    app = np.zeros(oc.n, dtype=np.float64)
    r = lib().or_decode_spa_grid(oc.handle, l, max_iter, hb.ctypes.data if hist else None,
                                 sy.ctypes.data, app.ctypes.data, int(early_stop), int(grid))
    out = dict(fail=r.fail, iters=r.iters, tmin=r.tmin, wmin=r.wmin, synd=sy[:r.iters], app=app)
    if hist:
        out["hist"] = hb[:r.iters]
    return out


def patterns(oc: OCode, kind: int) -> np.ndarray:
    L = lib()
    n = L.or_patterns(oc.handle, kind, None, 0)
    if n < 0:
        raise ValueError("bad pattern kind")
    out = np.zeros((n, kind), dtype=np.int32)
    L.or_patterns(oc.handle, kind, out.ctypes.data, n)
    return out


def pattern_list(oc: OCode, kinds) -> np.ndarray:
    """Concatenation of pattern families, padded with -1 to the widest."""
    parts = [patterns(oc, k) for k in kinds]
    w = max(p.shape[1] for p in parts)
    rows = [np.pad(p, ((0, 0), (0, w - p.shape[1])), constant_values=-1) for p in parts]
    return np.ascontiguousarray(np.concatenate(rows, axis=0).astype(np.int32))


def count_b(oc: OCode, s) -> int:
    a = _i32(s)
    return lib().or_count_b(oc.handle, a, a.size)


def tree(oc: OCode, s) -> np.ndarray:
    a = _i32(s)
    out = np.zeros(max(a.size, 1), dtype=np.int32)
    k = lib().or_tree(oc.handle, a, a.size, out)
    return out[:k].copy()


def ts_closure(oc: OCode, s, bound: int = 0) -> np.ndarray:
    a = _i32(s)
    out = np.zeros(a.size * (1 + 64 * 64) + 8 if not bound else bound, dtype=np.int32)
    k = lib().or_ts_closure(oc.handle, a, a.size, out)
    return out[:k].copy()


def canon(oc: OCode, s) -> Tuple[np.ndarray, int]:
    a = _i32(s)
    out = np.zeros(max(a.size, 1), dtype=np.int32)
    orb = C.c_int32()
    lib().or_canon(oc.handle, a, a.size, out, C.byref(orb))
    return out[:a.size].copy(), orb.value


@dataclass
class TsRecord:
    a: int
    b: int
    orbit: int
    first_pattern: int
    k_crit: int
    bits: Tuple[int, ...]


def search(oc: OCode, pats: np.ndarray, decoder: int = DEC_OMS, max_iter: int = 20,
           oms_offset: int = 1, ebn0_db: float = 3.0, rate: Optional[float] = None,
           llr_scale: float = 4.0, k_max: int = 512, k_den: int = 16, a_max: int = 6,
           extract_mode: int = EXTRACT_PATH, collect_from_iter: int = -1, threads: int = 0,
           spa_grid: int = 0):
    """spa_grid > 0 runs the conditioning probe of the sum-product decoder
    (or_decode_spa_grid): messages rounded to multiples of 2^-spa_grid."""
    pats = _i32(pats)
    if pats.ndim == 1:
        pats = pats.reshape(-1, 1)
    P, W = pats.shape
    rate = oc.code.rate if rate is None else rate
    o = SearchOpts(decoder, max_iter, oms_offset, ebn0_db, rate, llr_scale, k_max, k_den,
                   a_max, extract_mode, collect_from_iter, threads, spa_grid)
    kc, ic, il, tm, nc = (np.zeros(P, dtype=np.int32) for _ in range(5))
    dec, eu = C.c_int64(), C.c_int64()
    lst = C.c_void_p()
    L = lib()
    rc = L.or_search(oc.handle, C.byref(o), pats.ravel(), P, W, kc, ic, il, tm, nc,
                     C.byref(dec), C.byref(eu), C.byref(lst))
    if rc != 0:
        raise ValueError("oracle search rejected its options")
    recs: List[TsRecord] = []
    n = L.or_ts_count(lst)
    buf = np.zeros(max(a_max, 1), dtype=np.int32)
    a, b, orb, fp, k = (C.c_int32() for _ in range(5))
    for i in range(n):
        L.or_ts_get(lst, i, C.byref(a), C.byref(b), C.byref(orb), C.byref(fp), C.byref(k), buf)
        recs.append(TsRecord(a.value, b.value, orb.value, fp.value, k.value,
                             tuple(int(x) for x in buf[:a.value])))
    L.or_ts_free(lst)
    return dict(k_crit=kc, iters_crit=ic, iters_lo=il, tmin_crit=tm, n_cand=nc,
                decodes=dec.value, edge_updates=eu.value, ts=recs)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(c, k, out)
    return out


def normals(seed: int, frame: int, stream: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    lib().or_normals(seed, frame, stream, n, out)
    return out


IS_SPA, IS_LINEAR = 0, 1
IS_COUNT_ALL, IS_COUNT_TS = 0, 1


def is_estimate(oc: OCode, ts, ebn0_db: float, shift: float, n_frames: int, seed: int,
                frame_base: int = 0, stream: int = 0, max_iter: int = 50,
                rate: Optional[float] = None, threads: int = 0, want_fail: bool = False,
                decoder: int = IS_SPA, count_mode: int = 0, mix=None):
    """want_fail: "fail" = per-frame flags (bit 0 failed, bit 1 the set's own
    error event); count_mode IS_COUNT_TS counts only the latter.  mix = (m, s0,
    ds): the frames split over the m shifts s0 + k ds (balance heuristic)."""
    t = _i32(ts)
    rate = oc.code.rate if rate is None else rate
    m, s0, ds = mix if mix else (0, 0.0, 0.0)
    o = IsOpts(decoder, max_iter, ebn0_db, rate, shift, n_frames, seed, frame_base, stream,
               threads, count_mode, m, s0, ds)
    r = IsResult()
    fo = np.zeros(n_frames, dtype=np.uint8) if want_fail else None
    eu = C.c_int64()
    rc = lib().or_is_estimate(oc.handle, t, t.size, C.byref(o), C.byref(r),
                              fo.ctypes.data if want_fail else None, C.byref(eu))
    if rc != 0:
        raise ValueError("oracle IS rejected its options")
    out = {f: getattr(r, f) for f, _ in IsResult._fields_}
    out["edge_updates"] = eu.value
    if want_fail:
        out["fail"] = fo
    return out


def is_pilot_shift(oc: OCode, ts, ebn0_db: float, eps_star: float, pilot_frames: int, seed: int,
                   frame_base: int = 0, stream: int = 0, max_iter: int = 50,
                   rate: Optional[float] = None, threads: int = 0, count_mode: int = 0):
    """(chosen shift, relative variance of each of the 9 grid points, -1 where
    fewer than 10 counted failures)."""
    t = _i32(ts)
    rate = oc.code.rate if rate is None else rate
    o = IsOpts(IS_SPA, max_iter, ebn0_db, rate, 0.0, 2, seed, frame_base, stream, threads,
               count_mode, 0, 0.0, 0.0)
    rv = np.zeros(9, dtype=np.float64)
    s = lib().or_is_pilot_shift(oc.handle, t, t.size, C.byref(o), eps_star, pilot_frames, rv)
    return s, rv


def spa_eps_star(oc: OCode, ts, ebn0_db: float, max_iter: int = 50, eps_max: float = 32.0,
                 rate: Optional[float] = None) -> float:
    t = _i32(ts)
    rate = oc.code.rate if rate is None else rate
    return lib().or_spa_eps_star(oc.handle, t, t.size, ebn0_db, rate, max_iter, eps_max)


def brute_ts(oc: OCode, a_max: int, b_max: int = 32):
    counts = np.zeros((a_max + 1) * (b_max + 1), dtype=np.int64)
    orbits = np.zeros_like(counts)
    n = lib().or_brute_ts(oc.handle, a_max, b_max, counts, orbits)
    return n, counts.reshape(a_max + 1, b_max + 1), orbits.reshape(a_max + 1, b_max + 1)


def brute_ts_list(oc: OCode, a_max: int) -> List[Tuple[int, int, Tuple[int, ...]]]:
    L = lib()
    stride = 2 + a_max
    cap = 1 << 16
    while True:
        out = np.zeros(cap * stride, dtype=np.int32)
        n = L.or_brute_ts_list(oc.handle, a_max, out.ctypes.data, cap)
        if n <= cap:
            break
        cap = n
    out = out[:n * stride]
    out = out.reshape(n, stride)
    return [(int(r[0]), int(r[1]), tuple(int(x) for x in r[2:2 + r[0]])) for r in out]


def dmin(oc: OCode) -> Tuple[int, np.ndarray]:
    w = np.zeros(oc.n, dtype=np.int32)
    d = lib().or_dmin(oc.handle, w)
    return d, w[:max(d, 0)].copy()


def cycle_emd(oc: OCode, max_len: int = 8, emd_max: int = 32):
    L = lib()
    half = max_len // 2 + 1
    out = np.zeros(half * (emd_max + 1), dtype=np.int64)
    per_row = np.zeros(half * oc.code.mb, dtype=np.int64)
    per_col = np.zeros(half * oc.code.nb, dtype=np.int64)
    rc = L.or_cycle_emd(oc.handle, max_len, emd_max, out, per_row.ctypes.data,
                        per_col.ctypes.data)
    if rc != 0:
        raise ValueError("cycle counting needs a QC code")
    return (out.reshape(half, emd_max + 1), per_row.reshape(half, oc.code.mb),
            per_col.reshape(half, oc.code.nb))
