"""Frontier-centric BFS / SSSP for AMD Instinct MI355X (gfx950).

A thin ctypes binding over the ``gr_*`` C ABI declared in ``include/gr.h``:
argument marshalling only.  Every traversal step runs in the HIP kernels of
``libgr.so``; PyTorch provides device memory (output tensors) and streams.
There is no CPU fallback: without the built library or a gfx950 device the
calls raise.

Usage::

    import paper_1701_01170_amd as gr
    from paper_1701_01170_amd import graphgen
    hg = graphgen.add_weights(graphgen.rmat(14))
    ctx = gr.Context(0)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    depth, parent, stats = gr.bfs(g, source=3)
    dist, pred, stats = gr.sssp(g, [3])
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgr.so")

GR_OK, GR_EINVAL, GR_ERANGE, GR_ENOMEM, GR_EHIP, GR_ENODEV, GR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "GR_OK", -1: "GR_EINVAL", -2: "GR_ERANGE", -3: "GR_ENOMEM", -4: "GR_EHIP",
                -5: "GR_ENODEV", -6: "GR_EUNSUPPORTED"}
POLICY_HEURISTIC, POLICY_LEARNED, POLICY_FIXED, POLICY_RANDOM = 0, 1, 2, 3
PUSH_TWC, PUSH_LB, PULL_TWC, PULL_LB = 0, 1, 2, 3
ACTION_NAMES = ["PUSH_TWC", "PUSH_LB", "PULL_TWC", "PULL_LB"]
SYMMETRIC, DEVICE_INPUT, RENUMBER = 0x1, 0x2, 0x4
BFS_FILTER_AUTO, BFS_FILTER_ATOMIC, BFS_FILTER_IDEMPOTENT = 0, 1, 2
IDEM_CULL_WAVE, IDEM_CULL_HISTORY, IDEM_CULL_LABEL = 0x1, 0x2, 0x4
SSSP_OPT_CULL, SSSP_OPT_BINS = 0x1, 0x2
BC_DIR_AUTO, BC_DIR_PUSH, BC_DIR_PULL = 0, 1, 2
MLP_N_PARAMS = 1476


class GrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class LevelTrace(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("action", ctypes.c_int32),
                ("n_f", ctypes.c_int64), ("m_f", ctypes.c_int64), ("n_u", ctypes.c_int64),
                ("m_u", ctypes.c_int64), ("max_deg_f", ctypes.c_int64),
                ("features", ctypes.c_float * 8), ("step_us", ctypes.c_float),
                ("kernel_us", ctypes.c_float), ("kernel", ctypes.c_int32), ("n_next", ctypes.c_int64),
                ("n_in", ctypes.c_int64), ("inspected", ctypes.c_int64),
                ("n_cand", ctypes.c_int64)]


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("policy", ctypes.c_int32),
                ("fixed_action", ctypes.c_int32), ("lb_light_threshold", ctypes.c_int32),
                ("policy_seed", ctypes.c_uint64), ("do_a", ctypes.c_float), ("do_b", ctypes.c_float),
                ("lb_min_avg_degree", ctypes.c_float), ("max_iterations", ctypes.c_int32),
                ("lb_chunk", ctypes.c_int32), ("trace_capacity", ctypes.c_int32),
                ("trace", ctypes.POINTER(LevelTrace)), ("trace_count", ctypes.c_int32),
                ("device_max_edges", ctypes.c_int32), ("sssp_delta", ctypes.c_int32),
                ("learned_margin", ctypes.c_float), ("bfs_filter", ctypes.c_int32),
                ("idem_culls_off", ctypes.c_int32), ("idem_table_log2", ctypes.c_int32),
                ("adv_block", ctypes.c_int32), ("twc_wave_min", ctypes.c_int32),
                ("twc_block_min", ctypes.c_int32), ("graph_blocks", ctypes.c_int32),
                ("sssp_opt_off", ctypes.c_int32), ("sssp_multi_sweep", ctypes.c_int32),
                ("trace_steps_off", ctypes.c_int32), ("bc_dir", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("action_count", ctypes.c_int32 * 4),
                ("teps_edges", ctypes.c_int64), ("inspected_edges", ctypes.c_int64),
                ("device_ms", ctypes.c_float), ("pad", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return dict(iterations=self.iterations, action_count=list(self.action_count),
                    teps_edges=self.teps_edges, inspected_edges=self.inspected_edges,
                    device_ms=self.device_ms)


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("weighted", ctypes.c_int32), ("max_weight", ctypes.c_uint32),
                ("resorted", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p

# name -> (restype, argtypes); must cover every function of include/gr.h
_SIGNATURES = {
    "gr_abi_version": (ctypes.c_int32, []),
    "gr_abi_sizeof": (ctypes.c_int32, [ctypes.c_int32]),
    "gr_last_error": (ctypes.c_char_p, []),
    "gr_opts_default": (None, [ctypes.POINTER(Opts)]),
    "gr_ctx_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P)]),
    "gr_ctx_destroy": (ctypes.c_int, [_P]),
    "gr_ctx_set_policy": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "gr_validate_csr": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "gr_graph_from_csr": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P,
                                         ctypes.c_uint32, _P, ctypes.POINTER(_P)]),
    "gr_graph_free": (ctypes.c_int, [_P]),
    "gr_graph_get_info": (ctypes.c_int, [_P, ctypes.POINTER(GraphInfo)]),
    "gr_graph_export": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "gr_bfs": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                              ctypes.POINTER(RunStats)]),
    "gr_bfs_static": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                                     ctypes.POINTER(RunStats)]),
    "gr_sssp": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                               ctypes.POINTER(RunStats)]),
    "gr_bfs_multi": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                                    ctypes.POINTER(RunStats)]),
    "gr_sssp_multi": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                                     ctypes.POINTER(RunStats)]),
    "gr_bc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(Opts), _P,
                             ctypes.POINTER(RunStats)]),
    "gr_copy_bandwidth": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, _P,
                                         ctypes.POINTER(ctypes.c_float)]),
    "gr_mlp_forward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P]),
    "gr_mlp_loss_grad": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "gr_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
}


def lib() -> ctypes.CDLL:
    """Load libgr.so.  torch is imported first so that the process holds a
    single HIP runtime (torch's and the library's share one soname)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1701_01170_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        for which, cls in enumerate([Opts, RunStats, LevelTrace, GraphInfo]):
            if L.gr_abi_sizeof(which) != ctypes.sizeof(cls):
                raise RuntimeError(f"ABI layout mismatch for {cls.__name__}")
        _lib = L
    return _lib


def last_error() -> str:
    return (lib().gr_last_error() or b"").decode()


def check(rc: int) -> None:
    if rc != GR_OK:
        raise GrError(rc, last_error())


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().gr_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"gr_opts has no field {k}")
        setattr(o, k, v)
    return o


def _stream_handle(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


class Context:
    """One gr_ctx on a HIP device (owns the library's pooled scratch)."""

    def __init__(self, device: int = 0):
        h = _P()
        check(lib().gr_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)

    def set_policy(self, params) -> None:
        """Load selector MLP parameters (1476 float32: one network for every
        traversal; 2 x 1476: the single-source network, then the batched-BFS
        one) or None to unload."""
        if params is None:
            check(lib().gr_ctx_set_policy(self.handle, None, 0))
            return
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        check(lib().gr_ctx_set_policy(self.handle, p.ctypes.data, p.shape[0]))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().gr_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A CSR graph resident in device memory (gr_graph)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        info = GraphInfo()
        check(lib().gr_graph_get_info(handle, ctypes.byref(info)))
        self.n_vertices = info.n_vertices
        self.n_edges = info.n_edges
        self.max_degree = info.max_degree
        self.flags = info.flags
        self.weighted = bool(info.weighted)
        self.max_weight = info.max_weight
        self.resorted = bool(info.resorted)

    @classmethod
    def from_csr(cls, ctx: Context, row_offsets, col_indices, weights=None,
                 symmetric: bool = True, renumber: bool = False, stream=None) -> "Graph":
        """From host numpy arrays, or from device torch tensors."""
        import torch
        flags = (SYMMETRIC if symmetric else 0) | (RENUMBER if renumber else 0)
        if isinstance(row_offsets, torch.Tensor):
            flags |= DEVICE_INPUT
            R, C = row_offsets, col_indices
            W = weights
            V, E = R.numel() - 1, C.numel()
            ptrs = (R.data_ptr(), C.data_ptr() if E else None, None if W is None else W.data_ptr())
            keep = (R, C, W)
        else:
            R = np.ascontiguousarray(row_offsets, dtype=np.int32)
            C = np.ascontiguousarray(col_indices, dtype=np.int32)
            W = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
            V, E = R.shape[0] - 1, C.shape[0]
            if W is not None and E == 0:
                W = np.zeros(1, np.uint32)  # weighted graph without edges: any non-NULL pointer
            ptrs = (R.ctypes.data, C.ctypes.data if E else None,
                    None if W is None else W.ctypes.data)
            keep = (R, C, W)
        h = _P()
        st = _stream_handle(stream)
        rc = lib().gr_graph_from_csr(ctx.handle, V, E, ptrs[0], ptrs[1], ptrs[2], flags, st,
                                     ctypes.byref(h))
        del keep
        check(rc)
        return cls(ctx, h)

    @classmethod
    def from_host(cls, ctx: Context, hg, symmetric: bool = True, renumber: bool = False) -> "Graph":
        return cls.from_csr(ctx, hg.row_offsets, hg.col_indices, hg.weights, symmetric=symmetric,
                            renumber=renumber)

    def export(self, stream=None):
        """The ingested (sorted) CSR as device tensors (R, C, W or None)."""
        import torch
        dev = torch.device("cuda", self.ctx.device)
        R = torch.empty(self.n_vertices + 1, dtype=torch.int32, device=dev)
        C = torch.empty(max(self.n_edges, 1), dtype=torch.int32, device=dev)
        W = torch.empty(max(self.n_edges, 1), dtype=torch.int32, device=dev) if self.weighted else None
        check(lib().gr_graph_export(self.handle, _ptr(R), _ptr(C), _ptr(W), _stream_handle(stream)))
        return R, C[:self.n_edges], (None if W is None else W[:self.n_edges])

    def free(self) -> None:
        if getattr(self, "handle", None):
            lib().gr_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _opts_arg(opts):
    if opts is None:
        return None
    return ctypes.byref(opts)


def _empty(n, dtype, device):
    import torch
    return torch.empty(n, dtype=dtype, device=torch.device("cuda", device))


def bfs(g: Graph, source: int, want_parent: bool = True, opts: Opts | None = None, stream=None,
        out=None):
    """Single-source BFS.  Returns (depth int32[V], parent int32[V] or None,
    stats dict).  `out` may pass preallocated (depth, parent) tensors."""
    import torch
    if out is not None:
        depth, parent = out
    else:
        depth = _empty(g.n_vertices, torch.int32, g.ctx.device)
        parent = _empty(g.n_vertices, torch.int32, g.ctx.device) if want_parent else None
    st = RunStats()
    check(lib().gr_bfs(g.ctx.handle, g.handle, int(source), _ptr(depth), _ptr(parent),
                       _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return depth, parent, st.as_dict()


def bfs_static(g: Graph, source: int, out, opts: Opts | None = None, stream=None):
    """gr_bfs_static: BFS whose working arrays live in the library's static
    device workspace (no allocation inside the call).  `out` = (depth,
    parent or None), caller-allocated int32[V] tensors.  Returns stats."""
    depth, parent = out
    st = RunStats()
    check(lib().gr_bfs_static(g.ctx.handle, g.handle, int(source), _ptr(depth), _ptr(parent),
                              _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return st.as_dict()


STATIC_WORKSPACE_BYTES = 64 << 20


def sssp(g: Graph, sources, want_pred: bool = True, opts: Opts | None = None, stream=None,
         out=None):
    """Shortest paths from one or more sources.  Returns (dist uint32 values in
    an int32 tensor [V] (UINT32_MAX reads as -1), pred int32[V] or None,
    stats dict)."""
    import torch
    src = np.ascontiguousarray(np.asarray(sources).reshape(-1), dtype=np.int32)
    if out is not None:
        dist, pred = out
    else:
        dist = _empty(g.n_vertices, torch.int32, g.ctx.device)
        pred = _empty(g.n_vertices, torch.int32, g.ctx.device) if want_pred else None
    st = RunStats()
    check(lib().gr_sssp(g.ctx.handle, g.handle, src.ctypes.data, src.shape[0], _ptr(dist),
                        _ptr(pred), _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return dist, pred, st.as_dict()


def bfs_multi(g: Graph, sources, want_parent: bool = True, opts: Opts | None = None, stream=None,
              out=None):
    """k BFS runs sharing each graph sweep.  Returns (depth int32[k][V],
    parent int32[k][V] or None, stats dict)."""
    import torch
    src = np.ascontiguousarray(np.asarray(sources).reshape(-1), dtype=np.int32)
    k = src.shape[0]
    if out is not None:
        depth, parent = out
    else:
        depth = _empty(k * g.n_vertices, torch.int32, g.ctx.device).view(k, g.n_vertices)
        parent = (_empty(k * g.n_vertices, torch.int32, g.ctx.device).view(k, g.n_vertices)
                  if want_parent else None)
    st = RunStats()
    check(lib().gr_bfs_multi(g.ctx.handle, g.handle, src.ctypes.data, k, _ptr(depth), _ptr(parent),
                             _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return depth, parent, st.as_dict()


def sssp_multi(g: Graph, sources, want_pred: bool = True, opts: Opts | None = None, stream=None,
               out=None):
    """k single-source SSSP runs sharing each sweep (gr_sssp_multi).  Returns
    (dist int32[k][V] holding uint32 bits, pred int32[k][V] or None, stats)."""
    import torch
    src = np.ascontiguousarray(np.asarray(sources).reshape(-1), dtype=np.int32)
    k = int(src.shape[0])
    if out is not None:
        dist, pred = out
    else:
        dev = torch.device("cuda", g.ctx.device)
        dist = torch.empty((k, g.n_vertices), dtype=torch.int32, device=dev)
        pred = torch.empty((k, g.n_vertices), dtype=torch.int32, device=dev) if want_pred else None
    st = RunStats()
    check(lib().gr_sssp_multi(g.ctx.handle, g.handle, src.ctypes.data, k, _ptr(dist), _ptr(pred),
                              _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return dist, pred, st.as_dict()


def bc(g: Graph, sources, want_sigma: bool = False, opts: Opts | None = None, stream=None,
       out=None):
    """Betweenness centrality summed over `sources` (gr_bc).  Returns (bc
    float64[V], sigma float64[V] or None (one source only), stats dict)."""
    import torch
    src = np.ascontiguousarray(np.asarray(sources).reshape(-1), dtype=np.int32)
    if out is not None:
        b, sig = out
    else:
        dev = torch.device("cuda", g.ctx.device)
        b = torch.empty(g.n_vertices, dtype=torch.float64, device=dev)
        sig = torch.empty(g.n_vertices, dtype=torch.float64, device=dev) if want_sigma else None
    st = RunStats()
    check(lib().gr_bc(g.ctx.handle, g.handle, src.ctypes.data, int(src.shape[0]), _ptr(b), _ptr(sig),
                      _opts_arg(opts), _stream_handle(stream), ctypes.byref(st)))
    return b, sig, st.as_dict()


def mlp_forward(ctx: Context, params, X, stream=None):
    """Y[n][4] for device float32 tensors params[1476], X[n][8]."""
    import torch
    n = X.shape[0]
    Y = torch.empty((n, 4), dtype=torch.float32, device=X.device)
    check(lib().gr_mlp_forward(ctx.handle, _ptr(params), _ptr(X), n, _ptr(Y), _stream_handle(stream)))
    return Y


def mlp_loss_grad(ctx: Context, params, X, T, M, grad=None, loss=None, stream=None):
    """(grad[1476], loss[1]) device tensors for the masked MSE over X, T, M."""
    import torch
    if grad is None:
        grad = torch.empty(MLP_N_PARAMS, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check(lib().gr_mlp_loss_grad(ctx.handle, _ptr(params), _ptr(X), _ptr(T), _ptr(M), X.shape[0],
                                 _ptr(grad), _ptr(loss), _stream_handle(stream)))
    return grad, loss


def mlp_adam(ctx: Context, params, grad, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    """In-place Adam step on device tensors params, m, v (1-based step)."""
    check(lib().gr_mlp_adam(ctx.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step),
                            float(lr), float(beta1), float(beta2), float(eps),
                            _stream_handle(stream)))


def copy_bandwidth(ctx: Context, nbytes: int = 1 << 30, reps: int = 20, stream=None) -> float:
    """Measured HBM copy bandwidth in GB/s (read + write bytes per second)."""
    out = ctypes.c_float()
    check(lib().gr_copy_bandwidth(ctx.handle, int(nbytes), int(reps), _stream_handle(stream),
                                  ctypes.byref(out)))
    return float(out.value)


def u32(t):
    """View an int32 tensor holding uint32 values as int64 (for comparisons)."""
    return t.to(dtype=__import__("torch").int64) & 0xFFFFFFFF
