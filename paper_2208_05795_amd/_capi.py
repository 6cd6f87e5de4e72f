"""ctypes declarations of the C ABI in include/tsgpu.h (structures and prototypes)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsgpu.so")

TS_OK, TS_E_INVAL, TS_E_NOMEM, TS_E_DEVICE, TS_E_STATE, TS_E_BUSY, TS_E_TRUNC, TS_E_CANCELLED = \
    0, -1, -2, -3, -4, -5, -6, -7
TS_CODE_CSR, TS_CODE_QC = 1, 2
TS_PAT_SINGLES, TS_PAT_PAIRS, TS_PAT_TRIPLES = 1, 2, 3
TS_DEC_OMS_I8, TS_DEC_SPA_F32, TS_DEC_LNMS_Q4 = 0, 1, 2
TS_EXTRACT_PATH, TS_EXTRACT_CRITICAL = 0, 1
TS_MEM_HOST, TS_MEM_DEVICE = 0, 1
TS_LAYOUT_AUTO, TS_LAYOUT_REGISTER, TS_LAYOUT_STREAMED = 0, 1, 2
TS_LAYOUT_STREAMED_GATHER, TS_LAYOUT_STREAMED_ACCUM = 3, 4
TS_PAT_QC_ORBITS = 0x100
TS_IS_COUNT_ALL, TS_IS_COUNT_TS = 0, 1
TS_SHIFT_EPS, TS_SHIFT_PILOT, TS_SHIFT_MIX = 0, 1, 2
TS_JOB_SEARCH, TS_JOB_IS = 1, 2
TS_JOB_QUEUED, TS_JOB_RUNNING, TS_JOB_DONE, TS_JOB_CANCELLED = 0, 1, 2, 3

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class CtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("hip_stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", C.c_void_p), ("hbm_budget_bytes", C.c_size_t),
                ("rec_buffer_bytes", C.c_size_t)]


class CodeDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("m", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("mb", C.c_int32),
                ("nb", C.c_int32), ("z", C.c_int32), ("shifts", C.c_void_p)]


class CodeInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("e", C.c_int64), ("girth", C.c_int32),
                ("z", C.c_int32), ("dv_max", C.c_int32), ("dc_max", C.c_int32),
                ("n_layers", C.c_int32), ("streamed_qc", C.c_int32)]


class SearchOpts(C.Structure):
    _fields_ = [("decoder", C.c_int32), ("max_iter", C.c_int32), ("oms_offset", C.c_int32),
                ("ebn0_db", C.c_double), ("rate", C.c_double), ("llr_scale", C.c_double),
                ("k_max", C.c_int32), ("k_den", C.c_int32), ("a_max", C.c_int32),
                ("extract_mode", C.c_int32), ("collect_from_iter", C.c_int32), ("mem", C.c_int32),
                ("layout", C.c_int32), ("full_iterations", C.c_int32)]


class SearchOut(C.Structure):
    _fields_ = [("k_crit", C.c_void_p), ("iters_crit", C.c_void_p), ("iters_lo", C.c_void_p),
                ("tmin_crit", C.c_void_p), ("n_cand", C.c_void_p)]


class Record(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("orbit", C.c_int32),
                ("first_pattern", C.c_int32), ("k_crit", C.c_int32), ("reserved", C.c_int32),
                ("bits_off", C.c_int64)]


class IsOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("ebn0_db", C.c_double), ("rate", C.c_double),
                ("shift", C.c_double), ("n_frames", C.c_int64), ("seed", C.c_uint64),
                ("frame_base", C.c_uint64), ("stream", C.c_uint32), ("layout", C.c_int32),
                ("full_iterations", C.c_int32), ("count_mode", C.c_int32), ("shift_rule", C.c_int32),
                ("pilot_frames", C.c_int64)]


class IsResult(C.Structure):
    _fields_ = [("p_hat", C.c_double), ("var", C.c_double), ("ci_lo", C.c_double),
                ("ci_hi", C.c_double), ("sum_w", C.c_double), ("sum_w2", C.c_double),
                ("n", C.c_int64), ("n_fail", C.c_int64), ("shift_used", C.c_double)]


class UbOpts(C.Structure):
    _fields_ = [("n_ts", C.c_int32), ("n_snr", C.c_int32), ("ebn0_db", C.c_void_p),
                ("max_iter", C.c_int32), ("rate", C.c_double), ("shift", C.c_double),
                ("n_frames", C.c_int64), ("seed", C.c_uint64), ("layout", C.c_int32),
                ("count_mode", C.c_int32), ("shift_rule", C.c_int32), ("pilot_frames", C.c_int64)]


class UbPoint(C.Structure):
    _fields_ = [("ebn0_db", C.c_double), ("fer", C.c_double), ("var", C.c_double),
                ("ci_lo", C.c_double), ("ci_hi", C.c_double)]


class JobDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("code", C.c_void_p), ("search", SearchOpts),
                ("patterns", C.c_void_p), ("n_patterns", C.c_int32), ("width", C.c_int32),
                ("is_", IsOpts), ("ts_bits", C.c_void_p), ("a", C.c_int32)]


class JobInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("submit_ms", C.c_double),
                ("start_ms", C.c_double), ("end_ms", C.c_double), ("edge_updates", C.c_int64),
                ("device_bytes", C.c_int64), ("n_ts", C.c_int64), ("n_bits", C.c_int64),
                ("n_patterns", C.c_int32), ("reserved", C.c_int32), ("is_", IsResult)]


class Stats(C.Structure):
    _fields_ = [("decode_ms", C.c_double), ("extract_ms", C.c_double), ("total_ms", C.c_double),
                ("decodes", C.c_int64), ("edge_updates", C.c_int64), ("candidates", C.c_int64),
                ("decode_launches", C.c_int32), ("extract_launches", C.c_int32),
                ("block_threads", C.c_int32), ("grid_blocks", C.c_int32), ("layout", C.c_int32),
                ("checks_per_thread", C.c_int32)]


# name -> (restype, argtypes); every function of the header appears here
PROTOTYPES = {
    "ts_create": (C.c_int, [C.POINTER(CtxOpts), C.POINTER(C.c_void_p)]),
    "ts_destroy": (C.c_int, [C.c_void_p]),
    "ts_last_error": (C.c_char_p, []),
    "ts_load_code": (C.c_int, [C.c_void_p, C.POINTER(CodeDesc), C.POINTER(C.c_void_p)]),
    "ts_code_info": (C.c_int, [C.c_void_p, C.POINTER(CodeInfo)]),
    "ts_code_csr": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_free_code": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ts_make_patterns": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "ts_impulse_search": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SearchOpts), C.c_void_p,
                                    C.c_int32, C.c_int32, C.POINTER(SearchOut)]),
    "ts_collect": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                             C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "ts_reset_ts": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ts_is_estimate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(IsOpts), C.POINTER(IsResult), C.c_void_p]),
    "ts_is_estimate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                         C.POINTER(IsOpts), C.POINTER(IsResult), C.c_void_p]),
    "ts_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "ts_probe_lds": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "ts_cycle_emd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ts_spectrum": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "ts_union_bound": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(UbOpts), C.c_void_p, C.c_void_p]),
    "ts_serve_start": (C.c_int, [C.c_void_p, C.c_int32]),
    "ts_submit": (C.c_int, [C.c_void_p, C.POINTER(JobDesc), C.POINTER(C.c_uint64)]),
    "ts_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(JobInfo)]),
    "ts_job_outputs": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(SearchOut), C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_int64]),
    "ts_run_batch": (C.c_int, [C.c_void_p, C.POINTER(JobDesc), C.c_int32, C.POINTER(C.c_uint64)]),
    "ts_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ts_release": (C.c_int, [C.c_void_p, C.c_uint64]),
}


def load(path: str = LIB_PATH):
    """Loads the library and declares every prototype.  Raises if it is missing.

    torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    Importing torch first makes the dynamic linker bind this library to that
    already-loaded runtime, so the process holds one HIP runtime and torch's
    streams and allocations are valid here."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib
