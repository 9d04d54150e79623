"""Seeded synthetic graph generators shared by the GPU library's users, the
tests and the benchmark.

The module draws graphs, weights and sources only; it holds none of the
traversal arithmetic.  Workloads follow the paper's evaluation setup (Sec. 7,
dataset paragraph): R-MAT with edge factor 16 and initiator
a=0.57, b=0.19, c=0.19, d=0.05, undirected, no self-loops or duplicate edges,
SSSP weights uniform in 1..64.  The native part is ``graphgen.c`` (OpenMP,
counter-based random numbers, so results do not depend on the thread count).
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgrgen.so")
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int64),
        ("n_edges", ctypes.c_int64),
        ("row_offsets", ctypes.c_void_p),
        ("col_indices", ctypes.c_void_p),
    ]


def lib():
    """Load the native generator library (built by the package build step)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with "
                "`python -m paper_1701_01170_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        L.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_CSR)]
        L.gg_rmat.restype = ctypes.c_int
        L.gg_erdos_renyi.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                     ctypes.POINTER(_CSR)]
        L.gg_erdos_renyi.restype = ctypes.c_int
        L.gg_grid.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_CSR)]
        L.gg_grid.restype = ctypes.c_int
        L.gg_take.argtypes = [ctypes.POINTER(_CSR), ctypes.c_void_p, ctypes.c_void_p]
        L.gg_take.restype = None
        L.gg_free.argtypes = [ctypes.POINTER(_CSR)]
        L.gg_free.restype = None
        L.gg_weights.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.gg_weights.restype = None
        L.gg_sources.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_void_p]
        L.gg_sources.restype = ctypes.c_int64
        L.gg_hash3.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.gg_hash3.restype = ctypes.c_uint64
        _lib = L
    return _lib


@dataclasses.dataclass
class HostGraph:
    """An int32 CSR graph in host memory (row_offsets[V+1], col_indices[E],
    optional uint32 weights[E] aligned with col_indices)."""

    row_offsets: np.ndarray
    col_indices: np.ndarray
    weights: np.ndarray | None = None
    name: str = ""

    @property
    def n_vertices(self) -> int:
        return int(self.row_offsets.shape[0] - 1)

    @property
    def n_edges(self) -> int:
        return int(self.col_indices.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_offsets.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_offsets).tobytes())
        h.update(np.ascontiguousarray(self.col_indices).tobytes())
        if self.weights is not None:
            h.update(np.ascontiguousarray(self.weights).tobytes())
        return h.hexdigest()


def _take(csr: _CSR, rc: int, what: str) -> tuple[np.ndarray, np.ndarray]:
    if rc != 0:
        raise ValueError(f"{what}: generator returned {rc}")
    R = np.empty(csr.n_vertices + 1, dtype=np.int32)
    C = np.empty(max(csr.n_edges, 0), dtype=np.int32)
    lib().gg_take(ctypes.byref(csr), R.ctypes.data, C.ctypes.data if C.size else None)
    return R, C


def rmat(scale: int, edge_factor: float = 16, a: float = RMAT_A, b: float = RMAT_B,
         c: float = RMAT_C, seed: int = 1, permute: bool = True) -> HostGraph:
    """Undirected R-MAT graph (symmetrised, deduplicated, no self-loops)."""
    csr = _CSR()
    rc = lib().gg_rmat(int(scale), float(edge_factor), float(a), float(b), float(c),
                       int(seed) & 0xFFFFFFFFFFFFFFFF, 1 if permute else 0, ctypes.byref(csr))
    R, C = _take(csr, rc, "rmat")
    return HostGraph(R, C, name=f"rmat_s{scale}_e{edge_factor:g}_a{a:g}_seed{seed}")


def rmat_family(scale: int, edge_factor: float, a: float, seed: int = 1,
                permute: bool = True) -> HostGraph:
    """R-MAT with a varied `a`, keeping the paper's b:c:d = 0.19:0.19:0.05 ratio."""
    rest = 1.0 - a
    b = c = rest * 0.19 / 0.43
    return rmat(scale, edge_factor, a, b, c, seed=seed, permute=permute)


def erdos_renyi(n: int, avg_degree: float, seed: int = 1) -> HostGraph:
    csr = _CSR()
    rc = lib().gg_erdos_renyi(int(n), float(avg_degree), int(seed) & 0xFFFFFFFFFFFFFFFF,
                              ctypes.byref(csr))
    R, C = _take(csr, rc, "erdos_renyi")
    return HostGraph(R, C, name=f"er_n{n}_d{avg_degree:g}_seed{seed}")


def grid(rows: int, cols: int) -> HostGraph:
    """rows x cols 4-neighbour grid, row-major ids, no wrap-around."""
    csr = _CSR()
    rc = lib().gg_grid(int(rows), int(cols), ctypes.byref(csr))
    R, C = _take(csr, rc, "grid")
    return HostGraph(R, C, name=f"grid_{rows}x{cols}")


def add_weights(g: HostGraph, seed: int = 101, lo: int = 1, hi: int = 64) -> HostGraph:
    """Attach symmetric uint32 weights uniform in [lo, hi]."""
    W = np.empty(g.n_edges, dtype=np.uint32)
    if g.n_edges:
        lib().gg_weights(g.n_vertices, g.row_offsets.ctypes.data, g.col_indices.ctypes.data,
                         int(seed) & 0xFFFFFFFFFFFFFFFF, int(lo), int(hi), W.ctypes.data)
    g.weights = W
    return g


def sources(g: HostGraph, k: int, seed: int = 1000) -> np.ndarray:
    """k seeded sources, uniform over vertices of degree > 0."""
    out = np.empty(max(k, 0), dtype=np.int32)
    n = lib().gg_sources(g.n_vertices, g.row_offsets.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                         int(k), out.ctypes.data if out.size else None)
    if n == 0 and k > 0:
        raise ValueError("graph has no edges: no non-isolated source")
    return out


def from_edges(n_vertices: int, edges, weights=None, symmetric: bool = False) -> HostGraph:
    """CSR from an explicit directed edge list (kept in the given order per row;
    duplicates and self-loops are kept).  With symmetric=True every (u,v) also
    adds (v,u) with the same weight."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = None if weights is None else np.asarray(weights, dtype=np.uint32).reshape(-1)
    if symmetric:
        edges = np.concatenate([edges, edges[:, ::-1]], axis=0)
        if w is not None:
            w = np.concatenate([w, w])
    order = np.argsort(edges[:, 0], kind="stable")
    src = edges[order, 0]
    R = np.zeros(n_vertices + 1, dtype=np.int64)
    np.add.at(R, src + 1, 1)
    R = np.cumsum(R).astype(np.int32)
    C = edges[order, 1].astype(np.int32)
    W = None if w is None else w[order].astype(np.uint32)
    return HostGraph(R, C, W, name="edges")


def sort_adjacency(g: HostGraph) -> HostGraph:
    """Copy of g with each adjacency list sorted ascending (weights follow)."""
    V = g.n_vertices
    rows = np.repeat(np.arange(V, dtype=np.int64), g.degrees())
    order = np.lexsort((g.col_indices.astype(np.int64), rows))
    W = None if g.weights is None else g.weights[order]
    return HostGraph(g.row_offsets.copy(), g.col_indices[order].copy(), W, name=g.name)


def disjoint_union(graphs: list[HostGraph]) -> tuple[HostGraph, np.ndarray]:
    """Block-diagonal union of several graphs; returns the union and the vertex
    offset of each part (len = parts + 1)."""
    voff = np.zeros(len(graphs) + 1, dtype=np.int64)
    eoff = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        voff[i + 1] = voff[i] + g.n_vertices
        eoff[i + 1] = eoff[i] + g.n_edges
    if voff[-1] > np.iinfo(np.int32).max - 1 or eoff[-1] > np.iinfo(np.int32).max:
        raise ValueError("union exceeds int32 CSR limits")
    R = np.empty(voff[-1] + 1, dtype=np.int32)
    C = np.empty(eoff[-1], dtype=np.int32)
    have_w = all(g.weights is not None for g in graphs)
    W = np.empty(eoff[-1], dtype=np.uint32) if have_w else None
    for i, g in enumerate(graphs):
        R[voff[i]:voff[i + 1]] = g.row_offsets[:-1] + eoff[i]
        C[eoff[i]:eoff[i + 1]] = g.col_indices + voff[i]
        if have_w:
            W[eoff[i]:eoff[i + 1]] = g.weights
    R[-1] = eoff[-1]
    return HostGraph(R, C, W, name=f"union{len(graphs)}"), voff


def small_rmat_batch(n_graphs: int = 256, scale_lo: int = 10, scale_hi: int = 16,
                     ef_lo: int = 8, ef_hi: int = 32, seed: int = 7,
                     weight_seed: int = 101) -> tuple[list[HostGraph], np.ndarray]:
    """n_graphs R-MAT graphs with scale uniform in [scale_lo, scale_hi] and edge
    factor uniform in [ef_lo, ef_hi], each weighted; plus one seeded source per
    graph (local ids)."""
    L = lib()
    graphs, srcs = [], []
    for i in range(n_graphs):
        h = int(L.gg_hash3(seed, 11, i))
        s = scale_lo + (h % (scale_hi - scale_lo + 1))
        ef = ef_lo + ((h >> 20) % (ef_hi - ef_lo + 1))
        g = rmat(s, ef, seed=seed * 1000003 + i)
        add_weights(g, seed=weight_seed + i)
        graphs.append(g)
        srcs.append(int(sources(g, 1, seed=5000 + i)[0]))
    return graphs, np.asarray(srcs, dtype=np.int32)
