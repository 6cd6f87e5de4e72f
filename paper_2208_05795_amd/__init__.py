"""tsgpu: the trapping-set search of the modified Cole importance-sampling method
(arXiv 2208.05795) on AMD Instinct MI355X.

Thin Python binding over the C ABI of include/tsgpu.h: it only marshals
arguments.  Every step runs inside libtsgpu.so (HIP kernels for gfx950); PyTorch
provides device memory (its caching allocator) and the stream.  There is no CPU
fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _capi as A

__all__ = ["DEC_LNMS", "Context", "Code", "TsRecord", "TsgError", "DEC_OMS", "DEC_SPA",
           "PAT_SINGLES", "PAT_PAIRS", "PAT_TRIPLES", "EXTRACT_PATH", "EXTRACT_CRITICAL",
           "LAYOUT_AUTO", "LAYOUT_REGISTER", "LAYOUT_STREAMED", "LAYOUT_STREAMED_GATHER",
           "LAYOUT_STREAMED_ACCUM", "PAT_QC_ORBITS", "IS_COUNT_ALL", "IS_COUNT_TS", "SHIFT_EPS",
           "SHIFT_PILOT", "SHIFT_MIX"]

DEC_OMS, DEC_SPA, DEC_LNMS = A.TS_DEC_OMS_I8, A.TS_DEC_SPA_F32, A.TS_DEC_LNMS_Q4
PAT_SINGLES, PAT_PAIRS, PAT_TRIPLES = A.TS_PAT_SINGLES, A.TS_PAT_PAIRS, A.TS_PAT_TRIPLES
PAT_QC_ORBITS = A.TS_PAT_QC_ORBITS
EXTRACT_PATH, EXTRACT_CRITICAL = A.TS_EXTRACT_PATH, A.TS_EXTRACT_CRITICAL
IS_COUNT_ALL, IS_COUNT_TS = A.TS_IS_COUNT_ALL, A.TS_IS_COUNT_TS
SHIFT_EPS, SHIFT_PILOT, SHIFT_MIX = A.TS_SHIFT_EPS, A.TS_SHIFT_PILOT, A.TS_SHIFT_MIX
LAYOUT_AUTO, LAYOUT_REGISTER, LAYOUT_STREAMED = A.TS_LAYOUT_AUTO, A.TS_LAYOUT_REGISTER, A.TS_LAYOUT_STREAMED
LAYOUT_STREAMED_GATHER, LAYOUT_STREAMED_ACCUM = A.TS_LAYOUT_STREAMED_GATHER, A.TS_LAYOUT_STREAMED_ACCUM

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = A.load()
    return _lib


class TsgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tsgpu status {status}: {msg}")
        self.status = status


def _check(rc: int):
    if rc != A.TS_OK:
        raise TsgError(rc, lib().ts_last_error().decode(errors="replace"))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


@dataclass
class TsRecord:
    a: int
    b: int
    orbit: int
    first_pattern: int
    k_crit: int
    bits: Tuple[int, ...]


# numpy view of ts_record: a, b, orbit, first_pattern, k_crit, reserved, bits_off
_REC_DTYPE = np.dtype([("a", np.int32), ("b", np.int32), ("orbit", np.int32),
                       ("first_pattern", np.int32), ("k_crit", np.int32), ("reserved", np.int32),
                       ("bits_off", np.int64)])


def _ts_records(recs: np.ndarray, bits: np.ndarray) -> List[TsRecord]:
    # whole columns to Python lists first (per-row field access is slow)
    a, b, orb = recs["a"].tolist(), recs["b"].tolist(), recs["orbit"].tolist()
    fp, kc, off = recs["first_pattern"].tolist(), recs["k_crit"].tolist(), recs["bits_off"].tolist()
    bl = np.asarray(bits).tolist()
    return [TsRecord(a[i], b[i], orb[i], fp[i], kc[i], tuple(bl[off[i]:off[i] + a[i]]))
            for i in range(len(a))]


class Context:
    """A device, a stream and an allocator.  By default the stream and the
    allocator are torch's (current stream, caching allocator)."""

    def __init__(self, device: int = 0, torch_stream: bool = True, torch_alloc: bool = True,
                 hbm_budget_bytes: int = 0, rec_buffer_bytes: int = 0):
        L = lib()
        self._keep = []
        opts = A.CtxOpts()
        opts.device = device
        opts.hbm_budget_bytes = hbm_budget_bytes
        opts.rec_buffer_bytes = rec_buffer_bytes
        self.device = device
        if torch_stream or torch_alloc:
            import torch
            if not torch.cuda.is_available():
                raise TsgError(A.TS_E_DEVICE, "no GPU visible to torch")
            torch.cuda.set_device(device)
            if torch_stream:
                opts.hip_stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
            if torch_alloc:
                dev = device

                def _alloc(nbytes, user):
                    try:
                        return torch.cuda.caching_allocator_alloc(
                            int(nbytes), dev, torch.cuda.current_stream(dev))
                    except Exception:   # noqa: BLE001 - reported to C as NULL
                        return None

                def _free(ptr, user):
                    torch.cuda.caching_allocator_delete(ptr)

                fa, ff = A.ALLOC_FN(_alloc), A.FREE_FN(_free)
                self._keep += [fa, ff]
                opts.alloc = fa
                opts.free = ff
        h = C.c_void_p()
        _check(L.ts_create(C.byref(opts), C.byref(h)))
        self._h = h
        self._codes: List[Code] = []

    @property
    def handle(self):
        return self._h

    def load_code(self, code) -> "Code":
        return Code(self, code)

    # ---- serving -----------------------------------------------------------
    def serve_start(self, slots: int = 4):
        _check(lib().ts_serve_start(self._h, slots))

    @staticmethod
    def _search_desc(code: "Code", patterns, decoder: int = DEC_OMS, max_iter: int = 20,
                     oms_offset: int = 1, ebn0_db: float = 3.0, rate: Optional[float] = None,
                     llr_scale: float = 4.0, k_max: int = 512, k_den: int = 16, a_max: int = 6,
                     extract_mode: int = EXTRACT_PATH, collect_from_iter: int = -1,
                     layout: int = 0, full_iterations: bool = False):
        pats = _i32(patterns)
        if pats.ndim == 1:
            pats = pats.reshape(-1, 1)
        rate = (1.0 - code.m / code.n) if rate is None else rate
        d = A.JobDesc()
        d.kind, d.code = A.TS_JOB_SEARCH, code._h
        d.search = A.SearchOpts(decoder, max_iter, oms_offset, ebn0_db, rate, llr_scale, k_max,
                                k_den, a_max, extract_mode, collect_from_iter, A.TS_MEM_HOST,
                                layout, int(full_iterations))
        d.patterns, d.n_patterns, d.width = pats.ctypes.data, pats.shape[0], pats.shape[1]
        return d, pats

    @staticmethod
    def _is_desc(code: "Code", ts_bits, ebn0_db: float, shift: float, n_frames: int,
                 seed: int, frame_base: int = 0, stream: int = 0, max_iter: int = 50,
                 rate: Optional[float] = None, layout: int = 0, full_iterations: bool = False,
                 count_mode: int = IS_COUNT_ALL, shift_rule: int = SHIFT_EPS,
                 pilot_frames: int = 0):
        t = _i32(ts_bits)
        rate = (1.0 - code.m / code.n) if rate is None else rate
        d = A.JobDesc()
        d.kind, d.code = A.TS_JOB_IS, code._h
        d.is_ = A.IsOpts(max_iter, ebn0_db, rate, shift, n_frames, seed, frame_base, stream,
                         layout, int(full_iterations), count_mode, shift_rule, pilot_frames)
        d.ts_bits, d.a = t.ctypes.data, t.size
        return d, t

    def submit_search(self, code: "Code", patterns, **kw) -> int:
        """Queues a search job (arguments as Code.impulse_search); returns its id."""
        d, keep = self._search_desc(code, patterns, **kw)
        jid = C.c_uint64()
        _check(lib().ts_submit(self._h, C.byref(d), C.byref(jid)))
        return jid.value

    def submit_is(self, code: "Code", ts_bits, ebn0_db: float, shift: float, n_frames: int,
                  seed: int, **kw) -> int:
        """Queues an IS job (arguments as Code.is_estimate); returns its id."""
        d, keep = self._is_desc(code, ts_bits, ebn0_db, shift, n_frames, seed, **kw)
        jid = C.c_uint64()
        _check(lib().ts_submit(self._h, C.byref(d), C.byref(jid)))
        return jid.value

    def run_batch(self, jobs) -> List[int]:
        """Runs jobs as one batch (ts_run_batch).  jobs: ("search", code, patterns,
        kwargs) or ("is", code, ts_bits, kwargs) tuples; kwargs as for
        submit_search / submit_is.  Returns the job ids (finished jobs: read them
        with poll / job_outputs, free them with release)."""
        descs, keep = [], []
        for kind, code, data, kw in jobs:
            if kind == "search":
                d, k = self._search_desc(code, data, **kw)
            elif kind == "is":
                kw = dict(kw)
                d, k = self._is_desc(code, data, kw.pop("ebn0_db"), kw.pop("shift"),
                                     kw.pop("n_frames"), kw.pop("seed"), **kw)
            else:
                raise ValueError(f"unknown job kind {kind!r}")
            descs.append(d)
            keep.append(k)
        arr = (A.JobDesc * max(len(descs), 1))(*descs)
        ids = (C.c_uint64 * max(len(descs), 1))()
        _check(lib().ts_run_batch(self._h, arr, len(descs), ids))
        return [int(ids[i]) for i in range(len(descs))]

    def poll(self, job_id: int, wait: bool = False) -> dict:
        info = A.JobInfo()
        _check(lib().ts_poll(self._h, job_id, int(wait), C.byref(info)))
        out = {f: getattr(info, f) for f, _ in A.JobInfo._fields_ if f not in ("is_", "reserved")}
        out["is"] = {f: getattr(info.is_, f) for f, _ in A.IsResult._fields_}
        if info.state == A.TS_JOB_DONE and info.status != A.TS_OK:
            out["error"] = lib().ts_last_error().decode(errors="replace")
        return out

    def job_outputs(self, job_id: int, arrays: bool = False) -> dict:
        """Per-pattern outputs and the TS of a finished search job.  arrays=True
        gives the TS as a record array ("ts_recs", fields of ts_record) and the
        concatenated bits ("ts_bits"); otherwise "ts" is a list of TsRecord."""
        info = self.poll(job_id)
        P = info["n_patterns"]
        res = {k: np.zeros(P, dtype=np.int32)
               for k in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")}
        out = A.SearchOut(*(res[k].ctypes.data for k in
                            ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")))
        n, nb = info["n_ts"], info["n_bits"]
        recs = np.zeros(max(n, 1), dtype=_REC_DTYPE)
        bits = np.zeros(max(nb, 1), dtype=np.int32)
        _check(lib().ts_job_outputs(self._h, job_id, C.byref(out), recs.ctypes.data, n,
                                    bits.ctypes.data, nb))
        if arrays:
            res["ts_recs"], res["ts_bits"] = recs[:n], bits[:nb]
        else:
            res["ts"] = _ts_records(recs[:n], bits)
        return res

    def cancel(self, job_id: int):
        _check(lib().ts_cancel(self._h, job_id))

    def release(self, job_id: int):
        _check(lib().ts_release(self._h, job_id))

    def stats(self) -> dict:
        s = A.Stats()
        _check(lib().ts_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in A.Stats._fields_}

    def probe_lds(self) -> float:
        """LDS read bandwidth of the device in bytes/s (measurement aid)."""
        v = C.c_double()
        _check(lib().ts_probe_lds(self._h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            for c in list(self._codes):
                c._h = None
            lib().ts_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Code:
    """A parity-check matrix loaded on a context (QC or CSR form, see workloads.Code)."""

    def __init__(self, ctx: Context, code):
        self.ctx = ctx
        self.src = code
        d = A.CodeDesc()
        keep = []
        if code.kind == "qc":
            sh = _i32(code.shifts).ravel()
            keep.append(sh)
            d.kind, d.mb, d.nb, d.z = A.TS_CODE_QC, code.mb, code.nb, code.z
            d.shifts = sh.ctypes.data
        else:
            rp = np.ascontiguousarray(code.row_ptr, dtype=np.int64)
            col = _i32(code.col)
            keep += [rp, col]
            d.kind, d.n, d.m, d.nnz = A.TS_CODE_CSR, code.n, code.m, int(rp[-1])
            d.row_ptr, d.col_idx = rp.ctypes.data, col.ctypes.data
        h = C.c_void_p()
        _check(lib().ts_load_code(ctx.handle, C.byref(d), C.byref(h)))
        self._h = h
        ctx._codes.append(self)
        info = A.CodeInfo()
        _check(lib().ts_code_info(h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in A.CodeInfo._fields_}
        self.n, self.m, self.e = info.n, info.m, info.e
        self.girth, self.z = info.girth, info.z

    def csr(self):
        rp = np.zeros(self.m + 1, dtype=np.int64)
        col = np.zeros(self.e, dtype=np.int32)
        _check(lib().ts_code_csr(self._h, rp.ctypes.data, col.ctypes.data))
        return rp, col

    def make_patterns(self, kind: int) -> np.ndarray:
        n = C.c_int64()
        _check(lib().ts_make_patterns(self.ctx.handle, self._h, kind, None, 0, C.byref(n)))
        out = np.zeros((n.value, kind & 0xff), dtype=np.int32)
        _check(lib().ts_make_patterns(self.ctx.handle, self._h, kind, out.ctypes.data,
                                      n.value, C.byref(n)))
        return out

    def pattern_list(self, kinds: Sequence[int]) -> np.ndarray:
        parts = [self.make_patterns(k) for k in kinds]
        w = max(p.shape[1] for p in parts)
        rows = [np.pad(p, ((0, 0), (0, w - p.shape[1])), constant_values=-1) for p in parts]
        return np.ascontiguousarray(np.concatenate(rows, axis=0).astype(np.int32))

    def impulse_search(self, patterns, decoder: int = DEC_OMS, max_iter: int = 20,
                       oms_offset: int = 1, ebn0_db: float = 3.0, rate: Optional[float] = None,
                       llr_scale: float = 4.0, k_max: int = 512, k_den: int = 16, a_max: int = 6,
                       extract_mode: int = EXTRACT_PATH, collect_from_iter: int = -1,
                       layout: int = 0, full_iterations: bool = False) -> dict:
        """Patterns: numpy (host) or a torch int32 CUDA tensor [P, width] (device);
        outputs come back in the same kind of memory.  layout: LAYOUT_AUTO,
        LAYOUT_REGISTER, LAYOUT_STREAMED or one streamed variant
        (LAYOUT_STREAMED_GATHER, LAYOUT_STREAMED_ACCUM).  full_iterations: compute
        every iteration of every decode (no fixed-point exit; same results)."""
        rate = (1.0 - self.m / self.n) if rate is None else rate
        o = A.SearchOpts(decoder, max_iter, oms_offset, ebn0_db, rate, llr_scale, k_max, k_den,
                         a_max, extract_mode, collect_from_iter, A.TS_MEM_HOST, layout,
                         int(full_iterations))
        out = A.SearchOut()
        if _is_torch_cuda(patterns):
            import torch
            pats = patterns.contiguous()
            if pats.dtype != torch.int32 or pats.dim() != 2:
                raise ValueError("device patterns must be an int32 [P, width] tensor")
            P, W = pats.shape
            res = {k: torch.empty(P, dtype=torch.int32, device=pats.device)
                   for k in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")}
            o.mem = A.TS_MEM_DEVICE
            ptr = pats.data_ptr()
        else:
            pats = _i32(patterns)
            if pats.ndim == 1:
                pats = pats.reshape(-1, 1)
            P, W = pats.shape
            res = {k: np.zeros(P, dtype=np.int32)
                   for k in ("k_crit", "iters_crit", "iters_lo", "tmin_crit", "n_cand")}
            ptr = pats.ctypes.data

        def addr(x):
            return x.data_ptr() if o.mem == A.TS_MEM_DEVICE else x.ctypes.data

        out.k_crit, out.iters_crit = addr(res["k_crit"]), addr(res["iters_crit"])
        out.iters_lo, out.tmin_crit = addr(res["iters_lo"]), addr(res["tmin_crit"])
        out.n_cand = addr(res["n_cand"])
        _check(lib().ts_impulse_search(self.ctx.handle, self._h, C.byref(o), ptr, int(P), int(W),
                                       C.byref(out)))
        res["stats"] = self.ctx.stats()
        return res

    def collect_arrays(self):
        """The code's TS table in order: a record array (fields of ts_record) and
        the concatenated bits of the sets."""
        L = lib()
        n, nb = C.c_int64(), C.c_int64()
        _check(L.ts_collect(self.ctx.handle, self._h, None, 0, C.byref(n), None, 0, C.byref(nb)))
        recs = np.zeros(max(n.value, 1), dtype=_REC_DTYPE)
        bits = np.zeros(max(nb.value, 1), dtype=np.int32)
        _check(L.ts_collect(self.ctx.handle, self._h, recs.ctypes.data, n.value, C.byref(n),
                            bits.ctypes.data, nb.value, C.byref(nb)))
        return recs[:n.value], bits[:nb.value]

    def collect(self) -> List[TsRecord]:
        recs, bits = self.collect_arrays()
        return _ts_records(recs, bits)

    def cycle_emd(self, max_len: int = 8, emd_max: int = 32) -> np.ndarray:
        """counts[len // 2, emd] of simple cycles through the position-0 variable of
        each block column (ts_cycle_emd); an orbit of 2l-cycles adds l."""
        out = np.zeros((max_len // 2 + 1, emd_max + 1), dtype=np.int64)
        _check(lib().ts_cycle_emd(self.ctx.handle, self._h, max_len, emd_max, out.ctypes.data))
        return out

    def spectrum(self, a_max: int = 12, b_max: int = 16, by_orbit: bool = True) -> np.ndarray:
        """counts[a, b] of the TS table (ts_spectrum): canonical sets, or every set
        (orbit-weighted) when by_orbit is False."""
        out = np.zeros((a_max + 1, b_max + 1), dtype=np.int64)
        _check(lib().ts_spectrum(self.ctx.handle, self._h, a_max, b_max, int(by_orbit),
                                 out.ctypes.data))
        return out

    def union_bound(self, n_ts: int, ebn0_db, n_frames: int, seed: int, shift: float = -1.0,
                    max_iter: int = 50, rate: Optional[float] = None, layout: int = 0,
                    per_ts: bool = False, count_mode: int = IS_COUNT_ALL,
                    shift_rule: int = SHIFT_EPS, pilot_frames: int = 0) -> dict:
        """FER ~ sum over the first n_ts sets of the TS table of orbit x P_hat
        (ts_union_bound), one IS batch over all (set, SNR) pairs."""
        snr = np.ascontiguousarray(np.asarray(ebn0_db, dtype=np.float64).reshape(-1))
        rate = (1.0 - self.m / self.n) if rate is None else rate
        o = A.UbOpts(n_ts, snr.size, snr.ctypes.data, max_iter, rate, shift, n_frames, seed, layout,
                     count_mode, shift_rule, pilot_frames)
        pts = (A.UbPoint * snr.size)()
        rs = (A.IsResult * (snr.size * n_ts))() if per_ts else None
        _check(lib().ts_union_bound(self.ctx.handle, self._h, C.byref(o), pts, rs))
        out = {"points": [{f: getattr(p, f) for f, _ in A.UbPoint._fields_} for p in pts]}
        if per_ts:
            out["per_ts"] = [[{f: getattr(rs[i * n_ts + t], f) for f, _ in A.IsResult._fields_}
                              for t in range(n_ts)] for i in range(snr.size)]
        out["stats"] = self.ctx.stats()
        return out

    def reset_ts(self):
        _check(lib().ts_reset_ts(self.ctx.handle, self._h))

    def is_estimate(self, ts_bits, ebn0_db: float, shift: float, n_frames: int, seed: int,
                    frame_base: int = 0, stream: int = 0, max_iter: int = 50,
                    rate: Optional[float] = None, want_fail: bool = False,
                    layout: int = 0, full_iterations: bool = False,
                    count_mode: int = IS_COUNT_ALL, shift_rule: int = SHIFT_EPS,
                    pilot_frames: int = 0) -> dict:
        """want_fail: "fail" = per-frame flags (bit 0 the decode failed, bit 1 it
        failed with every bit of the set in error at the end)."""
        rate = (1.0 - self.m / self.n) if rate is None else rate
        t = _i32(ts_bits)
        o = A.IsOpts(max_iter, ebn0_db, rate, shift, n_frames, seed, frame_base, stream, layout,
                     int(full_iterations), count_mode, shift_rule, pilot_frames)
        r = A.IsResult()
        fo = np.zeros(n_frames, dtype=np.uint8) if want_fail else None
        _check(lib().ts_is_estimate(self.ctx.handle, self._h, t.ctypes.data, t.size, C.byref(o),
                                    C.byref(r), fo.ctypes.data if want_fail else None))
        out = {f: getattr(r, f) for f, _ in A.IsResult._fields_}
        out["stats"] = self.ctx.stats()
        if want_fail:
            out["fail"] = fo
        return out

    def free(self):
        if getattr(self, "_h", None) and self.ctx.handle:
            _check(lib().ts_free_code(self.ctx.handle, self._h))
            self.ctx._codes.remove(self)
        self._h = None
