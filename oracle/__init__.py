"""CPU oracle for frontier BFS / SSSP and for the strategy-selector MLP.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (its C part is ``oracle.c``, built by ``oracle/build.py``
with gcc; the MLP reference below is plain numpy in float64).

Graph results (definitions; see oracle.c for the full statement):
  * BC   (paper Sec. 6, betweenness centrality, Brandes's two passes):
    bc(v) = sum over the given sources s != v of the dependency delta_s(v),
    float64, no halving or normalisation.
  * BFS  (paper Sec. 6.1; labels / predecessors initialised as in Alg. 1,
    Set_Problem_Data): depth = fewest edges from the source (-1 unreached);
    parent = minimum-id in-neighbour one level closer (-1 for the source and
    for unreached vertices).
  * SSSP (paper Sec. 3 example, Sec. 6.2, Alg. 1 Update_Label): dist = minimum
    summed uint32 weight from any source (UINT32_MAX unreached); pred =
    minimum-id in-neighbour u with dist(u) + w(u,v) = dist(v) (-1 at sources
    and unreached vertices).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

UINT32_MAX = 0xFFFFFFFF


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401  (the oracle builds itself on demand)
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_bfs.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                             ctypes.c_void_p, ctypes.c_void_p]
        L.or_bfs.restype = ctypes.c_int
        L.or_sssp.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.or_sssp.restype = ctypes.c_int
        L.or_bc.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_bc.restype = ctypes.c_int
        _lib = L
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def bfs(row_offsets, col_indices, source: int, want_parent: bool = True):
    """Single-source BFS: returns (depth int32[V], parent int32[V] or None)."""
    R, C = _i32(row_offsets), _i32(col_indices)
    V = R.shape[0] - 1
    depth = np.empty(V, dtype=np.int32)
    parent = np.empty(V, dtype=np.int32) if want_parent else None
    rc = lib().or_bfs(V, R.ctypes.data, C.ctypes.data if C.size else None, int(source),
                      depth.ctypes.data, parent.ctypes.data if want_parent else None)
    if rc != 0:
        raise ValueError(f"oracle bfs failed ({rc})")
    return depth, parent


def bfs_multi(row_offsets, col_indices, sources, want_parent: bool = True):
    """K independent BFS runs: returns (depth int32[K][V], parent int32[K][V] or None)."""
    ds, ps = [], []
    for s in np.asarray(sources).reshape(-1):
        d, p = bfs(row_offsets, col_indices, int(s), want_parent)
        ds.append(d)
        ps.append(p)
    return np.stack(ds), (np.stack(ps) if want_parent else None)


def sssp(row_offsets, col_indices, weights, sources, want_pred: bool = True):
    """Multi-source Dijkstra: returns (dist uint32[V], pred int32[V] or None)."""
    R, C = _i32(row_offsets), _i32(col_indices)
    W = np.ascontiguousarray(weights, dtype=np.uint32)
    S = _i32(np.asarray(sources).reshape(-1))
    V = R.shape[0] - 1
    dist = np.empty(V, dtype=np.uint32)
    pred = np.empty(V, dtype=np.int32) if want_pred else None
    rc = lib().or_sssp(V, R.ctypes.data, C.ctypes.data if C.size else None,
                       W.ctypes.data if W.size else None, S.ctypes.data, S.shape[0],
                       dist.ctypes.data, pred.ctypes.data if want_pred else None)
    if rc == -2:
        raise OverflowError("a finite distance does not fit in uint32")
    if rc != 0:
        raise ValueError(f"oracle sssp failed ({rc})")
    return dist, pred


def bc(row_offsets, col_indices, sources, want_sigma: bool = False):
    """Betweenness centrality over the given sources (Brandes, float64; see
    or_bc in oracle.c for the definition): returns (bc float64[V], sigma of
    the last source float64[V] or None)."""
    R, C = _i32(row_offsets), _i32(col_indices)
    V = R.shape[0] - 1
    S = _i32(np.asarray(sources).reshape(-1))
    out = np.empty(V, dtype=np.float64)
    sig = np.empty(V, dtype=np.float64) if want_sigma else None
    rc = lib().or_bc(V, R.ctypes.data, C.ctypes.data if C.size else None, S.shape[0],
                     S.ctypes.data, out.ctypes.data, sig.ctypes.data if want_sigma else None)
    if rc != 0:
        raise ValueError(f"oracle bc failed ({rc})")
    return out, sig


def level_profile(row_offsets, depth):
    """Per-level frontier statistics of a finished BFS, straight from the
    definitions: for level d the frontier is {v : depth(v) = d}; n_f is its
    size, m_f the sum of its degrees, maxdeg its largest degree; n_u / m_u count
    the vertices (and their degrees) with depth > d or unreached."""
    R = np.asarray(row_offsets, dtype=np.int64)
    deg = np.diff(R)
    depth = np.asarray(depth)
    out = []
    n_levels = int(depth.max()) + 1 if depth.size and depth.max() >= 0 else 0
    for d in range(n_levels):
        f = depth == d
        u = (depth > d) | (depth < 0)
        out.append(dict(level=d, n_f=int(f.sum()), m_f=int(deg[f].sum()),
                        maxdeg_f=int(deg[f].max()) if f.any() else 0,
                        n_u=int(u.sum()), m_u=int(deg[u].sum())))
    return out


def teps_edges(row_offsets, reached_mask) -> int:
    """Sum of degrees over reached vertices (the paper's TEPS numerator, Sec. 7
    measurement methodology)."""
    deg = np.diff(np.asarray(row_offsets, dtype=np.int64))
    return int(deg[np.asarray(reached_mask)].sum())


# ---------------------------------------------------------------------------
# Strategy-selector MLP reference (float64).  Layers 8 -> 32 -> 32 -> 4 with
# ReLU on the two hidden layers; loss = masked mean squared error on the
# predicted log2 run time of each action; optimiser = Adam (Kingma & Ba 2015).
# ---------------------------------------------------------------------------

MLP_SHAPES = [("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)),
              ("W3", (4, 32)), ("b3", (4,))]
MLP_N_PARAMS = sum(int(np.prod(s)) for _, s in MLP_SHAPES)


def mlp_unflatten(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64).reshape(-1)
    if flat.shape[0] != MLP_N_PARAMS:
        raise ValueError(f"expected {MLP_N_PARAMS} parameters, got {flat.shape[0]}")
    out, o = {}, 0
    for name, shape in MLP_SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape).copy()
        o += n
    return out


def mlp_flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in MLP_SHAPES])


def mlp_forward(p: dict, X):
    """Returns (Y [N,4], cache)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    Y = h2 @ p["W3"].T + p["b3"]
    return Y, (X, z1, h1, z2, h2)


def mlp_loss(p: dict, X, T, M) -> float:
    Y, _ = mlp_forward(p, X)
    M = np.asarray(M, dtype=np.float64)
    denom = max(1.0, float(M.sum()))
    return float((M * (Y - np.asarray(T, dtype=np.float64)) ** 2).sum() / denom)


def mlp_backward(p: dict, X, T, M) -> tuple[float, dict]:
    """Loss and its gradient with respect to every parameter (chain rule
    written out layer by layer)."""
    Y, (X, z1, h1, z2, h2) = mlp_forward(p, X)
    M = np.asarray(M, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    denom = max(1.0, float(M.sum()))
    loss = float((M * (Y - T) ** 2).sum() / denom)
    dY = 2.0 * M * (Y - T) / denom
    g = {"W3": dY.T @ h2, "b3": dY.sum(0)}
    dh2 = dY @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(params: np.ndarray, grads: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update on flat float64 vectors; t is the 1-based step count.
    Returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
