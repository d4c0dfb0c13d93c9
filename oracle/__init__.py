"""CPU oracle for the dynamic random-walk transition sampler.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU implementation (``paper_2512_00705_amd``) and never imports it.

Two layers, both written from FlexiWalker (arXiv 2512.00705):

* ``exact`` -- the plain definition (Section 2.1, Eq. prob, Eq. node2vec, the
  MetaPath rule) in exact rational arithmetic, with brute-force enumeration of
  whole-path probabilities on tiny graphs.
* ``walk_oracle.c`` -- the canonical sample stream: eRVS with exponential keys and
  the jump (Section 3.2, Algorithm 1, Eq. jump), eRJS with the per-node bound
  (Section 3.3), the cost model (Section 4.1, Eq. runtime) and the helper estimates
  (Section 4.2, Eq. sum_estimation), driven by Philox4x32-10 (Salmon et al., SC'11)
  keyed by (seed; walker, step, draw, tag).  Plain sequential loops, float32
  arithmetic without contraction, logarithms in double rounded once to float32.

Parity of the canonical stream itself is a project definition; it is pinned to the
paper through the distribution tests in ``tests/`` (chi-square against ``exact``,
bound invariance of eRJS, jump equivalence of eRVS) and through published Philox
known answers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "walk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

AUTO, RVS_ONLY, RJS_ONLY, ITS, RANDOM_SELECT, DEGREE_SELECT = 0, 1, 2, 3, 4, 5
NODE2VEC, METAPATH, SECOND_PR = 1, 2, 3
COUNTER_NAMES = ("steps", "rjs_steps", "rvs_steps", "rjs_fallbacks", "rjs_trials", "rvs_triggers",
                 "ended_early", "alg_bytes", "flagged_steps")


class _Graph(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("ne", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("h", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("alias_thr", ctypes.c_void_p), ("alias_idx", ctypes.c_void_p), ("h8", ctypes.c_int32),
                ("nlab", ctypes.c_int32), ("lrow", ctypes.c_void_p), ("lperm", ctypes.c_void_p),
                ("lthr", ctypes.c_void_p), ("lalias", ctypes.c_void_p)]


class _Logic(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("weighted", ctypes.c_int32), ("p", ctypes.c_float),
                ("q", ctypes.c_float), ("gamma", ctypes.c_float), ("schema_len", ctypes.c_int32),
                ("schema", ctypes.c_uint8 * 64)]


class _Plan(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_float), ("d_lo", ctypes.c_int32), ("rjs_cap", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("jump", ctypes.c_int32), ("bound_scale", ctypes.c_float),
                ("bound", ctypes.c_int32), ("proposal", ctypes.c_int32), ("hub_deg", ctypes.c_int32),
                ("hub_lanes", ctypes.c_int32), ("rvs_share", ctypes.c_int32)]


@dataclass
class Logic:
    """Walk logic: Node2Vec (p = the paper's a, q = b), MetaPath (label schema) or
    second-order PageRank (gamma)."""
    kind: int = NODE2VEC
    weighted: bool = True
    p: float = 1.0
    q: float = 1.0
    schema: tuple = ()
    gamma: float = 0.2

    def _c(self):
        s = _Logic()
        s.kind, s.weighted, s.p, s.q = self.kind, int(self.weighted), self.p, self.q
        s.gamma = self.gamma
        s.schema_len = len(self.schema)
        for i, v in enumerate(self.schema):
            s.schema[i] = v
        return s


@dataclass
class Plan:
    """Parameters that change the sample stream (not only its speed)."""
    rho: float = 8.0
    d_lo: int = 0
    rjs_cap: int = 1024
    lanes: int = 64
    jump: bool = True
    bound_scale: float = 1.0
    bound: int = 0  # 0: max(w) * h_MAX (Section 3.3); 1: Node2Vec split bound (return edge apart)
    proposal: int = 0  # 0: uniform eRJS proposals (Section 3.3); 1: proportional to h (alias tables);
    # 2: as 1, and MetaPath proposes within the wanted label's group (label_alias)
    hub_deg: int = 0  # eRVS rows of at least this degree use hub_lanes lanes (0: never)
    hub_lanes: int = 64
    rvs_share: bool = False  # eRVS lanes take the largest threshold after each round with a jump event

    def _c(self):
        s = _Plan()
        s.rho, s.d_lo, s.rjs_cap, s.lanes = self.rho, self.d_lo, self.rjs_cap, self.lanes
        s.jump, s.bound_scale, s.bound = int(self.jump), self.bound_scale, self.bound
        s.proposal = self.proposal
        s.hub_deg, s.hub_lanes = self.hub_deg, self.hub_lanes
        s.rvs_share = int(self.rvs_share)
        return s


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no HIP headers, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    """Declare the C signatures on a loaded build of walk_oracle.c."""
    P = ctypes.c_void_p
    lib.og_philox.argtypes = [P, P, P]
    lib.og_philox.restype = None
    lib.og_uniform.argtypes = [ctypes.c_uint32]
    lib.og_uniform.restype = ctypes.c_float
    lib.og_preprocess.argtypes = [ctypes.POINTER(_Graph), P, P]
    lib.og_dequantize_h8.argtypes = [P, ctypes.c_float, ctypes.c_int64, P]
    lib.og_dequantize_h8.restype = None
    lib.og_build_alias.argtypes = [ctypes.POINTER(_Graph), P, P]
    lib.og_build_alias.restype = None
    lib.og_build_label_alias.argtypes = [ctypes.POINTER(_Graph), ctypes.c_int32, P, P, P, P]
    lib.og_build_label_alias.restype = ctypes.c_int
    lib.og_preprocess.restype = None
    lib.og_walk.argtypes = [ctypes.POINTER(_Graph), P, P, ctypes.POINTER(_Logic), ctypes.POINTER(_Plan),
                            ctypes.c_int, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                            P, P, P, P, P, ctypes.c_int]
    lib.og_walk.restype = ctypes.c_int
    lib.og_step_once.argtypes = [ctypes.POINTER(_Graph), P, P, ctypes.POINTER(_Logic), ctypes.POINTER(_Plan),
                                 ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, P, P, P, P]
    lib.og_step_once.restype = ctypes.c_int32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def build_variant(path: str, defines: dict) -> str:
    """Compile the oracle with extra -D macros (used by tests that plant a mistake)."""
    flags = [f"-D{k}={v}" for k, v in defines.items()]
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
                           "-shared", "-fPIC", *flags, _SRC, "-o", path, "-lm"])
    return path


class use_library:
    """Context manager: route every oracle call through another build of walk_oracle.c."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self.saved = _lib
        _lib = _configure(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


class Graph:
    """CSR view for the C oracle; keeps the numpy arrays alive."""

    def __init__(self, g: dict):
        self.nv, self.ne = int(g["nv"]), int(g["ne"])
        self.row_ptr = np.ascontiguousarray(g["row_ptr"], np.int64)
        self.col = np.ascontiguousarray(g["col"], np.int32)
        self.h = None if g.get("h") is None else np.ascontiguousarray(g["h"], np.float32)
        if g.get("h8") is not None:  # 8-bit property weights: h = h_scale * code
            assert self.h is None, "give h or h8, not both"
            self.h = dequantize_h8(g["h8"], g["h_scale"])
        self.label = None if g.get("label") is None else np.ascontiguousarray(g["label"], np.uint8)
        s = _Graph()
        s.nv, s.ne = self.nv, self.ne
        s.row_ptr, s.col = self.row_ptr.ctypes.data, self.col.ctypes.data
        s.h = self.h.ctypes.data if self.h is not None else None
        s.label = self.label.ctypes.data if self.label is not None else None
        s.h8 = int(g.get("h8") is not None)
        self._s = s
        self._aux = None
        self._alias = None
        self._label_alias = None

    def aux(self):
        """(h_MAX, h_SUM) per node, computed by the oracle."""
        if self._aux is None:
            hmax = np.empty(self.nv, np.float32)
            hsum = np.empty(self.nv, np.float32)
            _load().og_preprocess(ctypes.byref(self._s), hmax.ctypes.data, hsum.ctypes.data)
            self._aux = (hmax, hsum)
        return self._aux

    def alias(self):
        """(threshold, alias offset) per CSR entry: the alias tables of the static weights h
        used by h-proportional eRJS proposals (og_build_alias)."""
        if self._alias is None:
            thr = np.empty(max(self.ne, 1), np.uint32)
            idx = np.empty(max(self.ne, 1), np.int32)
            _load().og_build_alias(ctypes.byref(self._s), thr.ctypes.data, idx.ctypes.data)
            self._alias = (thr, idx)
            self._s.alias_thr, self._s.alias_idx = thr.ctypes.data, idx.ctypes.data
        return self._alias

    def label_alias(self):
        """(nlab, lrow, lperm, lthr, lalias): the label groups of each row and their alias
        tables, used by label-conditioned MetaPath proposals (og_build_label_alias); nlab is
        the largest label + 1."""
        if self._label_alias is None:
            assert self.label is not None, "label-conditioned proposals need edge labels"
            nlab = int(self.label.max()) + 1 if self.ne > 0 else 1
            lrow = np.empty(self.nv * nlab + 1, np.int64)
            lperm = np.empty(max(self.ne, 1), np.int32)
            lthr = np.empty(max(self.ne, 1), np.uint32)
            lalias = np.empty(max(self.ne, 1), np.int32)
            rc = _load().og_build_label_alias(ctypes.byref(self._s), nlab, lrow.ctypes.data, lperm.ctypes.data,
                                              lthr.ctypes.data, lalias.ctypes.data)
            assert rc == 0
            self._label_alias = (nlab, lrow, lperm, lthr, lalias)
            self._s.nlab = nlab
            self._s.lrow, self._s.lperm = lrow.ctypes.data, lperm.ctypes.data
            self._s.lthr, self._s.lalias = lthr.ctypes.data, lalias.ctypes.data
        return self._label_alias


def dequantize_h8(code, h_scale: float) -> np.ndarray:
    """Weights of 8-bit codes: h = h_scale * code in float32 (og_dequantize_h8)."""
    c = np.ascontiguousarray(code, np.uint8)
    out = np.empty(c.shape[0], np.float32)
    _load().og_dequantize_h8(c.ctypes.data, float(np.float32(h_scale)), c.shape[0], out.ctypes.data)
    return out


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key -> 4 x uint32."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.empty(4, np.uint32)
    _load().og_philox(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def uniform(x: int) -> float:
    return float(_load().og_uniform(ctypes.c_uint32(int(x) & 0xFFFFFFFF)))


@dataclass
class WalkResult:
    paths: np.ndarray
    lengths: np.ndarray
    margins: np.ndarray | None
    kinds: np.ndarray | None
    counters: dict = field(default_factory=dict)


def _tables(graph: Graph, logic: Logic, plan: Plan):
    """Build the proposal tables a plan reads: the alias tables for h-proportional
    proposals, and the label groups for label-conditioned MetaPath proposals."""
    if plan.proposal == 2 and logic.kind == METAPATH:
        graph.label_alias()
    elif plan.proposal:
        graph.alias()


def walk(graph: Graph, logic: Logic, plan: Plan, strategy: int, starts, L: int, seed: int,
         walker_ids=None, diagnostics: bool = True, nthreads: int = 0) -> WalkResult:
    """Free-running walks from ``starts`` (see ``og_walk`` in walk_oracle.c)."""
    lib = _load()
    starts = np.ascontiguousarray(starts, np.int32)
    n = starts.shape[0]
    wid = None if walker_ids is None else np.ascontiguousarray(walker_ids, np.int64)
    hmax, hsum = graph.aux()
    _tables(graph, logic, plan)
    paths = np.empty((n, L + 1), np.int32)
    lengths = np.empty(n, np.int32)
    margins = np.empty((n, L), np.float32) if diagnostics else None
    kinds = np.empty((n, L), np.int8) if diagnostics else None
    ctr = np.zeros(len(COUNTER_NAMES), np.float64)
    lg, pl = logic._c(), plan._c()
    rc = lib.og_walk(ctypes.byref(graph._s), hmax.ctypes.data, hsum.ctypes.data, ctypes.byref(lg),
                     ctypes.byref(pl), strategy, starts.ctypes.data,
                     wid.ctypes.data if wid is not None else None, n, L, seed, paths.ctypes.data,
                     lengths.ctypes.data, margins.ctypes.data if margins is not None else None,
                     kinds.ctypes.data if kinds is not None else None, ctr.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("og_walk: start vertex out of range")
    return WalkResult(paths, lengths, margins, kinds, dict(zip(COUNTER_NAMES, ctr.tolist())))


def step_info(graph: Graph, logic: Logic, plan: Plan, strategy: int, seed: int, walker: int, j: int,
              prev: int, cur: int) -> dict:
    """One transition from (prev, cur) at step j: the next vertex (-1: the walk ends), the
    smallest relative margin of its float decisions, its kind (0 eRVS, 1 eRJS, 2 eRJS capped
    then eRVS, 3 ITS, -1 ended), its eRJS trials and its algorithmic bytes."""
    lib = _load()
    hmax, hsum = graph.aux()
    _tables(graph, logic, plan)
    m = ctypes.c_float()
    k = ctypes.c_int32()
    t = ctypes.c_int32()
    b = ctypes.c_double()
    lg, pl = logic._c(), plan._c()
    r = lib.og_step_once(ctypes.byref(graph._s), hmax.ctypes.data, hsum.ctypes.data, ctypes.byref(lg),
                         ctypes.byref(pl), strategy, seed, walker, j, prev, cur, ctypes.byref(m),
                         ctypes.byref(k), ctypes.byref(t), ctypes.byref(b))
    return {"next": int(r), "margin": float(m.value), "kind": int(k.value), "trials": int(t.value),
            "bytes": float(b.value)}


def step_once(graph: Graph, logic: Logic, plan: Plan, strategy: int, seed: int, walker: int, j: int,
              prev: int, cur: int):
    """One transition from (prev, cur) at step j; returns (next, margin, kind, trials)."""
    r = step_info(graph, logic, plan, strategy, seed, walker, j, prev, cur)
    return r["next"], r["margin"], r["kind"], r["trials"]
