"""CPU-side checks of the C ABI: the library loads, exports every function that
include/gr.h declares, struct layouts agree with the binding, and host-side
validation returns the documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1701_01170_amd as gr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "gr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gr_[a-z0-9_]+)\s*\(", src)))


def test_library_loads_and_version():
    L = gr.lib()
    assert L.gr_abi_version() == 6


def test_every_declared_symbol_is_exported_and_bound():
    L = gr.lib()
    names = header_functions()
    assert "gr_bfs" in names and "gr_sssp" in names and "gr_bfs_multi" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in gr.h but not exported"
    assert sorted(gr._SIGNATURES) == names


def test_struct_sizes():
    L = gr.lib()
    assert L.gr_abi_sizeof(0) == ctypes.sizeof(gr.Opts)
    assert L.gr_abi_sizeof(1) == ctypes.sizeof(gr.RunStats)
    assert L.gr_abi_sizeof(2) == ctypes.sizeof(gr.LevelTrace)
    assert L.gr_abi_sizeof(3) == ctypes.sizeof(gr.GraphInfo)
    assert L.gr_abi_sizeof(99) == -1


def test_opts_default():
    o = gr.default_opts()
    assert o.struct_size == ctypes.sizeof(gr.Opts)
    assert o.policy == gr.POLICY_HEURISTIC
    assert o.lb_light_threshold == 4096
    assert abs(o.lb_min_avg_degree - 5.0) < 1e-6
    assert abs(o.do_a - 1 / 14) < 1e-6 and abs(o.do_b - 1 / 576) < 1e-7


def validate(R, C, V=None, E=None):
    R = np.ascontiguousarray(R, dtype=np.int32)
    C = np.ascontiguousarray(C, dtype=np.int32)
    V = R.shape[0] - 1 if V is None else V
    E = C.shape[0] if E is None else E
    return gr.lib().gr_validate_csr(V, E, R.ctypes.data, C.ctypes.data if C.size else None)


def test_validate_csr_codes():
    assert validate([0, 2, 3], [1, 0, 0]) == gr.GR_OK
    assert validate([0], []) == gr.GR_ERANGE                    # V = 0
    assert validate([1, 2, 3], [1, 0, 0]) == gr.GR_EINVAL        # R[0] != 0
    assert validate([0, 2, 1], [1, 0]) == gr.GR_EINVAL           # decreasing
    assert validate([0, 2, 2], [1, 0, 0]) == gr.GR_EINVAL        # R[V] != E
    assert validate([0, 2, 3], [1, 2, 0]) == gr.GR_EINVAL        # col out of range
    assert validate([0, 2, 3], [1, -1, 0]) == gr.GR_EINVAL       # negative col
    assert "out of range" in gr.last_error()
    assert validate([0, 0, 0], [], E=2 ** 31) == gr.GR_ERANGE    # E too large
    L = gr.lib()
    assert L.gr_validate_csr(2, 0, None, None) == gr.GR_EINVAL  # NULL row offsets


def test_graph_from_csr_validates_before_device():
    L = gr.lib()
    R = np.array([0, 2, 1], np.int32)
    C = np.array([1, 0], np.int32)
    h = ctypes.c_void_p()
    rc = L.gr_graph_from_csr(None, 2, 2, R.ctypes.data, C.ctypes.data, None, 1, None, ctypes.byref(h))
    assert rc == gr.GR_EINVAL and not h.value
    R = np.array([0, 1, 2], np.int32)
    C = np.array([1, 0], np.int32)
    rc = L.gr_graph_from_csr(None, 2, 2, R.ctypes.data, C.ctypes.data, None, 0x100, None,
                             ctypes.byref(h))
    assert rc == gr.GR_EINVAL and "flags" in gr.last_error()
    rc = L.gr_graph_from_csr(None, 2, 2, R.ctypes.data, C.ctypes.data, None, 1, None, ctypes.byref(h))
    assert rc == gr.GR_EINVAL and "ctx" in gr.last_error()


def test_traversal_argument_checks_without_device():
    L = gr.lib()
    st = gr.RunStats()
    assert L.gr_bfs(None, None, 0, None, None, None, None, ctypes.byref(st)) == gr.GR_EINVAL
    src = np.zeros(1, np.int32)
    assert L.gr_sssp(None, None, src.ctypes.data, 1, None, None, None, None, None) == gr.GR_EINVAL
    assert L.gr_bfs_multi(None, None, src.ctypes.data, 1, None, None, None, None, None) != gr.GR_OK


def test_ctx_create_without_gpu_is_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert gr.lib().gr_ctx_create(0, ctypes.byref(h)) == gr.GR_ENODEV
    with pytest.raises(gr.GrError) as ei:
        gr.Context(0)
    assert ei.value.code == gr.GR_ENODEV
