"""Python binding of libflexiwalk.so, the MI355X dynamic random-walk sampler.

Argument marshalling only: every step of the walk runs in the HIP kernels behind the
C ABI declared in ``include/flexiwalk.h``.  The functions keep the C names.  Pointer
arguments accept a torch tensor (its ``data_ptr()``), a numpy array (host memory), a
plain integer address or ``None``.  ``stream`` defaults to torch's current stream.

There is no fallback: importing the package without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflexiwalk.so")

FW_OK, FW_E_INVALID, FW_E_NOMEM, FW_E_DEVICE, FW_E_STATE, FW_E_BUSY = 0, 1, 2, 3, 4, 5
FW_AUTO, FW_RVS_ONLY, FW_RJS_ONLY, FW_RANDOM_SELECT, FW_DEGREE_SELECT = 0, 1, 2, 4, 5
FW_NODE2VEC, FW_METAPATH, FW_SECOND_PR = 1, 2, 3
FW_MAX_SCHEMA = 64
FW_NOALLOC_MAX_QUERIES = 4096
FW_NSTATS = 8
STAT_NAMES = ("steps", "rjs_steps", "rvs_steps", "rjs_fallbacks", "rjs_trials", "rvs_triggers",
              "ended_early", "alg_bytes")
EXPORTED = ("fw_graph_create", "fw_graph_destroy", "fw_graph_preprocess", "fw_graph_build_index",
            "fw_graph_export_aux", "fw_graph_export_alias", "fw_graph_info", "fw_calibrate_random_reads", "fw_graph_build_alias", "fw_graph_build_label_alias",
            "fw_logic_node2vec", "fw_logic_metapath", "fw_logic_second_pr", "fw_plan_default", "fw_plan_profile",
            "fw_plan_autotune", "fw_plan_autotune_mix", "fw_walk", "fw_graph_check", "fw_last_error", "fw_batch_create", "fw_batch_launch",
            "fw_batch_capture", "fw_batch_replay", "fw_batch_destroy", "fw_batch_run_noalloc", "fw_server_create",
            "fw_server_submit",
            "fw_server_next_done", "fw_server_result", "fw_server_stats", "fw_server_destroy")
SERVER_STAT_NAMES = ("waiting", "active", "finished", "ticks", "walker_steps", "bytes_in_use", "peak_bytes",
                     "alg_bytes")


class FlexiWalkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[fw status {code}] {msg}")
        self.code = code


class fw_csr(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("ne", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("h", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("on_device", ctypes.c_int32), ("h8", ctypes.c_void_p), ("h_scale", ctypes.c_float)]


class fw_logic(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("weighted", ctypes.c_int32), ("p", ctypes.c_float),
                ("q", ctypes.c_float), ("gamma", ctypes.c_float), ("schema_len", ctypes.c_int32),
                ("schema", ctypes.c_uint8 * FW_MAX_SCHEMA)]


class fw_plan(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_float), ("d_lo", ctypes.c_int32), ("rjs_cap", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("lds_cap", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("bound", ctypes.c_int32), ("proposal", ctypes.c_int32), ("hub_deg", ctypes.c_int32),
                ("hub_lanes", ctypes.c_int32), ("rvs_share", ctypes.c_int32)]


class fw_query(ctypes.Structure):
    _fields_ = [("logic", fw_logic), ("n", ctypes.c_int64), ("L", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("start_off", ctypes.c_int64), ("out_off", ctypes.c_int64), ("len_off", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2512_00705_amd._build` "
                           "(or __graft_entry__.build()) first. There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "fw_graph_create": ([ctypes.POINTER(fw_csr), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "fw_graph_destroy": ([P], ctypes.c_int),
        "fw_graph_preprocess": ([P, P], ctypes.c_int),
        "fw_graph_build_index": ([P, P], ctypes.c_int),
        "fw_graph_build_alias": ([P, P], ctypes.c_int),
        "fw_graph_build_label_alias": ([P, P], ctypes.c_int),
        "fw_calibrate_random_reads": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
        "fw_graph_export_aux": ([P, P, P], ctypes.c_int),
        "fw_graph_export_alias": ([P, P, P], ctypes.c_int),
        "fw_graph_info": ([P, P, P, P, P], ctypes.c_int),
        "fw_logic_node2vec": ([ctypes.c_float, ctypes.c_float, I32, ctypes.POINTER(fw_logic)], ctypes.c_int),
        "fw_logic_metapath": ([P, I32, I32, ctypes.POINTER(fw_logic)], ctypes.c_int),
        "fw_logic_second_pr": ([ctypes.c_float, I32, ctypes.POINTER(fw_logic)], ctypes.c_int),
        "fw_plan_default": ([ctypes.POINTER(fw_plan)], ctypes.c_int),
        "fw_plan_profile": ([P, ctypes.POINTER(fw_logic), ctypes.POINTER(fw_plan), P], ctypes.c_int),
        "fw_plan_autotune": ([P, ctypes.POINTER(fw_logic), ctypes.POINTER(fw_plan), P], ctypes.c_int),
        "fw_plan_autotune_mix": ([P, ctypes.POINTER(fw_logic), ctypes.c_int32, ctypes.POINTER(fw_plan), P],
                                 ctypes.c_int),
        "fw_walk": ([P, ctypes.POINTER(fw_logic), ctypes.POINTER(fw_plan), I32, P, I64, I32, ctypes.c_uint64,
                     P, P, P, P], ctypes.c_int),
        "fw_graph_check": ([P, P], ctypes.c_int),
        "fw_batch_create": ([P, ctypes.POINTER(fw_query), I64, ctypes.POINTER(fw_plan), I32, P, I64, P, I64, P,
                             I64, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "fw_batch_launch": ([P, P, P], ctypes.c_int),
        "fw_batch_capture": ([P, P, P], ctypes.c_int),
        "fw_batch_replay": ([P, P], ctypes.c_int),
        "fw_batch_destroy": ([P], ctypes.c_int),
        "fw_batch_run_noalloc": ([P, P, I64, ctypes.POINTER(fw_plan), I32, P, I64, P, I64, P, I64, P, P],
                                 ctypes.c_int),
        "fw_server_create": ([P, ctypes.POINTER(fw_plan), I32, ctypes.c_uint64, I32, I32, I32,
                              ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "fw_server_submit": ([P, ctypes.POINTER(fw_logic), P, I64, I32, ctypes.c_uint64,
                              ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "fw_server_next_done": ([P, I32, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "fw_server_result": ([P, ctypes.c_uint64, P, P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "fw_server_stats": ([P, P], ctypes.c_int),
        "fw_server_destroy": ([P], ctypes.c_int),
        "fw_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def _check(rc: int):
    if rc != FW_OK:
        raise FlexiWalkError(rc, _lib.fw_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x)} as a pointer")


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else getattr(stream, "cuda_stream", stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def fw_last_error() -> str:
    return _lib.fw_last_error().decode()


def fw_graph_create(nv: int, ne: int, row_ptr, col, h=None, label=None, on_device: bool = False, h8=None,
                    h_scale: float = 0.0) -> int:
    """Returns an opaque graph handle (int).  Arrays: numpy (host) or torch (device).
    ``h8``/``h_scale``: 8-bit property weights h = h_scale * code instead of ``h``."""
    c = fw_csr(nv, ne, _ptr(row_ptr), _ptr(col), _ptr(h), _ptr(label), int(on_device), _ptr(h8), float(h_scale))
    out = ctypes.c_void_p()
    _check(_lib.fw_graph_create(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def fw_graph_destroy(g: int):
    _check(_lib.fw_graph_destroy(g))


def fw_graph_preprocess(g: int, stream=None):
    _check(_lib.fw_graph_preprocess(g, _stream(stream)))


def fw_graph_build_index(g: int, stream=None):
    _check(_lib.fw_graph_build_index(g, _stream(stream)))


def fw_graph_build_alias(g: int, stream=None):
    _check(_lib.fw_graph_build_alias(g, _stream(stream)))


def fw_graph_build_label_alias(g: int, stream=None):
    _check(_lib.fw_graph_build_label_alias(g, _stream(stream)))


def fw_calibrate_random_reads(nbytes: int = 4 << 30, stream=None) -> float:
    """Random 8-byte reads per second the device sustains over an array of ``nbytes``."""
    out = ctypes.c_double()
    _check(_lib.fw_calibrate_random_reads(int(nbytes), ctypes.byref(out), _stream(stream)))
    return out.value


def fw_graph_export_alias(g: int, ne: int):
    """(thr uint32[ne], alias int32[ne]) of the proposal records' alias tables."""
    thr = np.empty(ne, np.uint32)
    alias = np.empty(ne, np.int32)
    _check(_lib.fw_graph_export_alias(g, thr.ctypes.data, alias.ctypes.data))
    return thr, alias


def fw_graph_export_aux(g: int, nv: int):
    hmax = np.empty(nv, np.float32)
    hsum = np.empty(nv, np.float32)
    _check(_lib.fw_graph_export_aux(g, hmax.ctypes.data, hsum.ctypes.data))
    return hmax, hsum


def fw_graph_info(g: int):
    """(nv, ne, max_deg, symmetric)"""
    nv, ne, md, sym = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.fw_graph_info(g, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(md), ctypes.byref(sym)))
    return nv.value, ne.value, md.value, bool(sym.value)


def fw_logic_node2vec(p: float, q: float, weighted: bool = True) -> fw_logic:
    out = fw_logic()
    _check(_lib.fw_logic_node2vec(p, q, int(weighted), ctypes.byref(out)))
    return out


def fw_logic_metapath(schema, weighted: bool = True) -> fw_logic:
    arr = np.ascontiguousarray(np.asarray(schema, dtype=np.uint8))
    out = fw_logic()
    _check(_lib.fw_logic_metapath(arr.ctypes.data, len(arr), int(weighted), ctypes.byref(out)))
    return out


def fw_logic_second_pr(gamma: float, weighted: bool = True) -> fw_logic:
    out = fw_logic()
    _check(_lib.fw_logic_second_pr(float(gamma), int(weighted), ctypes.byref(out)))
    return out


def fw_plan_default(**overrides) -> fw_plan:
    out = fw_plan()
    _check(_lib.fw_plan_default(ctypes.byref(out)))
    for k, v in overrides.items():
        setattr(out, k, v)
    return out


def fw_plan_profile(g: int, logic: fw_logic, stream=None) -> fw_plan:
    out = fw_plan()
    _check(_lib.fw_plan_profile(g, ctypes.byref(logic), ctypes.byref(out), _stream(stream)))
    return out


def fw_plan_autotune(g: int, logic: fw_logic, stream=None) -> fw_plan:
    out = fw_plan()
    _check(_lib.fw_plan_autotune(g, ctypes.byref(logic), ctypes.byref(out), _stream(stream)))
    return out


def fw_plan_autotune_mix(g: int, logics, stream=None) -> fw_plan:
    """One plan for a mix of logics (a batch or a server's requests)."""
    arr = (fw_logic * len(logics))(*logics)
    out = fw_plan()
    _check(_lib.fw_plan_autotune_mix(g, arr, len(logics), ctypes.byref(out), _stream(stream)))
    return out


def fw_walk(g: int, logic: fw_logic, plan: fw_plan, strategy: int, starts, n: int, L: int, seed: int, paths,
            lengths, stats=None, stream=None):
    """Asynchronous on ``stream``; pointers are device pointers (torch tensors)."""
    _check(_lib.fw_walk(g, ctypes.byref(logic), ctypes.byref(plan), strategy, _ptr(starts), n, L,
                        seed & 0xFFFFFFFFFFFFFFFF, _ptr(paths), _ptr(lengths), _ptr(stats), _stream(stream)))


def fw_graph_check(g: int, stream=None):
    _check(_lib.fw_graph_check(g, _stream(stream)))


def _numel(x, given):
    if given is not None:
        return int(given)
    if x is None:
        return 0
    return int(x.numel()) if hasattr(x, "numel") else int(np.asarray(x).size)


def fw_batch_create(g: int, queries, plan: fw_plan, strategy: int, starts, paths, lengths, starts_len=None,
                    paths_len=None, lengths_len=None) -> int:
    """queries: a sequence of fw_query.  Array lengths default to the tensors' sizes.
    Returns an opaque batch handle (int)."""
    arr = (fw_query * max(len(queries), 1))(*queries)
    out = ctypes.c_void_p()
    _check(_lib.fw_batch_create(g, arr, len(queries), ctypes.byref(plan), strategy, _ptr(starts),
                                _numel(starts, starts_len), _ptr(paths), _numel(paths, paths_len), _ptr(lengths),
                                _numel(lengths, lengths_len), ctypes.byref(out)))
    return out.value


def fw_batch_launch(b: int, stats=None, stream=None):
    _check(_lib.fw_batch_launch(b, _ptr(stats), _stream(stream)))


def fw_batch_capture(b: int, stats=None, stream=None):
    _check(_lib.fw_batch_capture(b, _ptr(stats), _stream(stream)))


def fw_batch_replay(b: int, stream=None):
    _check(_lib.fw_batch_replay(b, _stream(stream)))


def fw_batch_destroy(b: int):
    _check(_lib.fw_batch_destroy(b))


def fw_batch_run_noalloc(g: int, queries, plan: fw_plan, strategy: int, starts, paths, lengths, stats=None,
                         stream=None, starts_len=None, paths_len=None, lengths_len=None):
    """fw_batch_create + fw_batch_launch in one call that allocates no device memory."""
    arr = (fw_query * max(len(queries), 1))(*queries)
    _check(_lib.fw_batch_run_noalloc(g, arr, len(queries), ctypes.byref(plan), strategy, _ptr(starts),
                                     _numel(starts, starts_len), _ptr(paths), _numel(paths, paths_len),
                                     _ptr(lengths), _numel(lengths, lengths_len), _ptr(stats), _stream(stream)))


def fw_server_create(g: int, plan: fw_plan, strategy: int, hbm_budget: int, tick_steps: int = 16,
                     max_active: int = 4096, max_pending: int = 1 << 16) -> int:
    out = ctypes.c_void_p()
    _check(_lib.fw_server_create(g, ctypes.byref(plan), strategy, hbm_budget, tick_steps, max_active, max_pending,
                                 ctypes.byref(out)))
    return out.value


def fw_server_submit(s: int, logic: fw_logic, starts, L: int, seed: int) -> int:
    """starts: host int32 array (copied).  Returns the request id."""
    st = np.ascontiguousarray(starts, dtype=np.int32)
    rid = ctypes.c_uint64()
    _check(_lib.fw_server_submit(s, ctypes.byref(logic), st.ctypes.data, st.shape[0], L,
                                 seed & 0xFFFFFFFFFFFFFFFF, ctypes.byref(rid)))
    return rid.value


def fw_server_next_done(s: int, timeout_ms: int = 100) -> int:
    rid = ctypes.c_uint64()
    _check(_lib.fw_server_next_done(s, timeout_ms, ctypes.byref(rid)))
    return rid.value


def fw_server_result(s: int, req_id: int, n: int, L: int):
    """(paths (n, L+1), lengths (n,), latency seconds) of a finished request."""
    paths = np.empty((n, L + 1), np.int32)
    lengths = np.empty(n, np.int32)
    lat = ctypes.c_double()
    _check(_lib.fw_server_result(s, req_id, paths.ctypes.data, lengths.ctypes.data, ctypes.byref(lat)))
    return paths, lengths, lat.value


def fw_server_stats(s: int) -> dict:
    out = np.zeros(8, np.uint64)
    _check(_lib.fw_server_stats(s, out.ctypes.data))
    return dict(zip(SERVER_STAT_NAMES, (int(x) for x in out)))


def fw_server_destroy(s: int):
    _check(_lib.fw_server_destroy(s))
