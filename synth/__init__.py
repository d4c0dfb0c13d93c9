"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *produces inputs* (graphs, edge properties, start vertices).  It
contains none of the random-walk arithmetic, so sharing it does not couple the
oracle to the GPU implementation.

Graphs are R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004), the standard stand-in
for the social/web graphs a random-walk paper evaluates on: undirected, self-loops
dropped, duplicates merged, vertex ids shuffled by a seeded permutation, rows
sorted ascending, ``int64`` row pointers, ``int32`` column indices, ``float32``
property weights and ``uint8`` labels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "librmat.so")
_lib = None


class _CSR(ctypes.Structure):
    _fields_ = [
        ("nv", ctypes.c_int64),
        ("ne", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("h", ctypes.POINTER(ctypes.c_float)),
        ("label", ctypes.POINTER(ctypes.c_uint8)),
    ]


def build(force: bool = True) -> str:
    """Compile the generator with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.synth_rmat.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint64, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(_CSR),
        ]
        lib.synth_rmat.restype = ctypes.c_int
        lib.synth_free.argtypes = [ctypes.POINTER(_CSR)]
        lib.synth_free.restype = None
        lib.synth_edge_props.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
            ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.synth_edge_props.restype = ctypes.c_int
        _lib = lib
    return _lib


def rmat(scale: int, ndraws: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True, weighted: bool = True, wlo: float = 1.0,
         whi: float = 10.0, nlabels: int = 0) -> dict:
    """Undirected R-MAT graph with ``2**scale`` vertices from ``ndraws`` edge draws.

    Returns a dict with ``nv, ne, row_ptr (i64), col (i32), h (f32 or None),
    label (u8 or None)``.
    """
    lib = _load()
    out = _CSR()
    rc = lib.synth_rmat(scale, ndraws, a, b, c, seed, int(permute), wlo, whi, max(nlabels, 1),
                        int(weighted), int(nlabels > 0), ctypes.byref(out))
    if rc != 0:
        raise MemoryError("synth_rmat: allocation failed")
    try:
        nv, ne = out.nv, out.ne
        g = {
            "nv": nv,
            "ne": ne,
            "row_ptr": np.ctypeslib.as_array(out.row_ptr, shape=(nv + 1,)).copy(),
            "col": np.ctypeslib.as_array(out.col, shape=(max(ne, 1),))[:ne].copy(),
            "h": np.ctypeslib.as_array(out.h, shape=(max(ne, 1),))[:ne].copy() if weighted else None,
            "label": np.ctypeslib.as_array(out.label, shape=(max(ne, 1),))[:ne].copy() if nlabels > 0 else None,
        }
    finally:
        lib.synth_free(ctypes.byref(out))
    return g


def edge_props(row_ptr: np.ndarray, col: np.ndarray, seed: int, wlo: float = 1.0, whi: float = 10.0,
               nlabels: int = 0, want_h: bool = True):
    """Hashed per-edge weights U[wlo, whi) and labels U{0..nlabels-1} for an existing CSR."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    h = np.empty(col.shape[0], np.float32) if want_h else None
    lab = np.empty(col.shape[0], np.uint8) if nlabels > 0 else None
    lib.synth_edge_props(row_ptr.shape[0] - 1, row_ptr.ctypes.data, col.ctypes.data, seed, wlo, whi,
                         max(nlabels, 1), h.ctypes.data if h is not None else None,
                         lab.ctypes.data if lab is not None else None)
    return h, lab


def pareto_weights(row_ptr: np.ndarray, col: np.ndarray, alpha: float, seed: int) -> np.ndarray:
    """Power-law property weights as numpy.random.pareto draws them (Lomax: (1 - U)^(-1/alpha) - 1),
    with U hashed from the unordered vertex pair so both directions of an edge agree."""
    u, _ = edge_props(row_ptr, col, seed, 0.0, 1.0)
    return ((1.0 - u.astype(np.float64)) ** (-1.0 / alpha) - 1.0).astype(np.float32)


def degree_weights(row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Property weight of edge (v, u) = d(u), the neighbouring vertex's degree (not symmetric)."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    return deg[np.asarray(col)].astype(np.float32)


def quantize_u8(h: np.ndarray, h_top: float = 10.0) -> tuple[np.ndarray, np.float32]:
    """8-bit codes for float weights in (0, h_top]: scale = h_top / 255 in float32 and
    code = clip(round(h / scale), 1, 255), so U(1, 10) weights become codes 25..255.
    Returns (codes uint8, scale); the weights such a graph carries are scale * code."""
    scale = np.float32(h_top / 255.0)
    c = np.rint(np.asarray(h, np.float64) / np.float64(scale))
    return np.clip(c, 1, 255).astype(np.uint8), scale


def csr_from_edges(nv: int, edges, h=None, label=None, symmetric: bool = True) -> dict:
    """Small hand-built graphs: CSR from an edge list with optional per-edge values.

    With ``symmetric`` each (u, v) is stored in both directions with the same value.
    Rows come out sorted; duplicate edges are rejected.
    """
    rows = [[] for _ in range(nv)]
    for k, (u, v) in enumerate(edges):
        hv = None if h is None else float(h[k])
        lv = None if label is None else int(label[k])
        rows[u].append((v, hv, lv))
        if symmetric and u != v:
            rows[v].append((u, hv, lv))
    row_ptr = np.zeros(nv + 1, np.int64)
    cols, hs, ls = [], [], []
    for v in range(nv):
        r = sorted(rows[v], key=lambda t: t[0])
        if len({t[0] for t in r}) != len(r):
            raise ValueError(f"duplicate edge in row {v}")
        row_ptr[v + 1] = row_ptr[v] + len(r)
        cols += [t[0] for t in r]
        hs += [t[1] for t in r]
        ls += [t[2] for t in r]
    return {
        "nv": nv,
        "ne": int(row_ptr[-1]),
        "row_ptr": row_ptr,
        "col": np.array(cols, np.int32),
        "h": None if h is None else np.array(hs, np.float32),
        "label": None if label is None else np.array(ls, np.uint8),
    }


def uniform_starts(nv: int, n: int, seed: int) -> np.ndarray:
    """``n`` start vertices drawn uniformly with replacement (numpy PCG64)."""
    return np.random.Generator(np.random.PCG64(seed)).integers(0, nv, size=n, dtype=np.int64).astype(np.int32)


def all_vertices(nv: int) -> np.ndarray:
    """One walker per vertex, in vertex order."""
    return np.arange(nv, dtype=np.int32)


# --- named workloads -------------------------------------------------------------
# R-MAT (a, b, c) = (0.57, 0.19, 0.19), d = 0.05; graph seed 1; weights U(1, 10).

def cached(name: str, cache_dir: str | None = None) -> dict:
    """``workload_graph(name)`` memoised as an uncompressed .npz under ``cache_dir``
    (default ``$FLEXIWALK_CACHE`` or /tmp/flexiwalk_cache)."""
    d = cache_dir or os.environ.get("FLEXIWALK_CACHE", "/tmp/flexiwalk_cache")
    path = os.path.join(d, f"{name}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        g = {k: z[k] for k in z.files}
        g["nv"], g["ne"] = int(g["nv"]), int(g["ne"])
        g.setdefault("h", None)
        g.setdefault("label", None)
        return g
    g = workload_graph(name)
    os.makedirs(d, exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, **{k: v for k, v in g.items() if v is not None})
    os.replace(tmp, path)
    return g


def batch_queries(nv: int, nq: int, seed: int, n_max: int = 65536, L_lo: int = 5, L_hi: int = 200,
                  pq=(0.25, 0.5, 1.0, 2.0, 4.0), first_seed: int = 42) -> dict:
    """A batch of Node2Vec walk queries.

    Per query: p and q drawn independently from ``pq``; start-set size
    ``floor(exp(U(0, ln n_max)))`` (log-uniform in 1..n_max); length uniform in
    L_lo..L_hi; seed ``first_seed + query index``; start vertices uniform over all
    vertices.  Returns arrays ``p, q, n, L, seed`` per query, the concatenated
    ``starts`` and the offsets ``start_off, out_off, len_off`` of each query's blocks.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.choice(np.asarray(pq, np.float32), nq)
    q = rng.choice(np.asarray(pq, np.float32), nq)
    n = np.floor(np.exp(rng.uniform(0.0, np.log(n_max), nq))).astype(np.int64)
    n = np.clip(n, 1, n_max)
    L = rng.integers(L_lo, L_hi + 1, nq).astype(np.int32)
    starts = rng.integers(0, nv, int(n.sum()), dtype=np.int64).astype(np.int32)
    start_off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(n * (L.astype(np.int64) + 1))[:-1]]).astype(np.int64)
    return {"p": p, "q": q, "n": n, "L": L, "seed": first_seed + np.arange(nq, dtype=np.int64),
            "starts": starts, "start_off": start_off, "out_off": out_off, "len_off": start_off.copy(),
            "total_paths": int((n * (L.astype(np.int64) + 1)).sum())}


def workload_graph(name: str) -> dict:
    """Graphs of the named workloads.

    * ``rmat12``: scale 12, average degree 16 (8 * 2^12 undirected draws).
    * ``rmat22``: scale 22, edge factor 16 (16 * 2^22 draws, <= 134M entries).
    * ``rmat22_labels``: the scale-22 graph plus uint8 labels uniform in 0..4.
    * ``rmat24_skew``: scale 24, edge factor 16, heavier skew (a, b, c) = (0.6, 0.175,
      0.175).
    * ``rmat25_labels``: scale 25, edge factor 16 (~1.07 B entries), labels 0..4.
    """
    if name == "rmat12":
        return rmat(12, 8 << 12, seed=1)
    if name == "rmat22":
        return rmat(22, 16 << 22, seed=1)
    if name == "rmat22_labels":
        return rmat(22, 16 << 22, seed=1, nlabels=5)
    if name == "rmat25_labels":
        return rmat(25, 16 << 25, seed=1, nlabels=5)
    if name == "rmat24_skew":
        return rmat(24, 16 << 24, a=0.6, b=0.175, c=0.175, seed=1)
    if name.startswith("rmat") and name[4:].isdigit():
        s = int(name[4:])
        return rmat(s, 16 << s, seed=1)
    raise KeyError(name)
