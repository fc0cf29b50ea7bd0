"""C ABI contract on the CPU: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1806_11558_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hm.h")).read()
    decl = r"^(?:hm_status|void|const char\*)\s+(hm_\w+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = hm.lib()
    names = _declared()
    assert {"hm_build", "hm_matvec", "hm_matvec_T", "hm_solve", "hm_free"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_struct_sizes_match_header():
    assert ctypes.sizeof(hm.Params) == 40
    assert ctypes.sizeof(hm.SolveParams) == 40
    assert ctypes.sizeof(hm.SolveInfo) == 24
    assert ctypes.sizeof(hm.Stats) == 21 * 8


def test_defaults():
    p = hm.hm_params_default()
    assert (p.leaf_size, p.max_rank, p.precision, p.eta, p.aca_eps) == (32, 64, hm.HM_F64, 1.0, 1e-6)


def _tri():
    return np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 2]])


@pytest.mark.parametrize("field,value", [
    ("leaf_size", 0), ("leaf_size", 65), ("max_rank", -1), ("max_rank", 257),
    ("precision", 7), ("eta", -1.0), ("eta", float("inf")), ("aca_eps", -1e-3),
    ("aca_eps", float("nan")), ("mem_limit_bytes", -5), ("flags", 16), ("flags", 32)])
def test_invalid_params_rejected(field, value):
    V, T = _tri()
    p = hm.hm_params_default()
    setattr(p, field, value)
    with pytest.raises(hm.HMError) as e:
        hm.hm_build(V, T, p, stream=0)
    assert e.value.status == -1


@pytest.mark.parametrize("V,T,what", [
    (np.zeros((3, 3)), np.array([[0, 1, 2]]), "degenerate"),
    (np.eye(3), np.array([[0, 1, 3]]), "out of range"),
    (np.eye(3), np.array([[0, -1, 2]]), "out of range"),
    (np.array([[0.0, 0, 0], [1, 0, 0], [np.nan, 1, 0]]), np.array([[0, 1, 2]]), "non-finite"),
    (np.eye(3), np.zeros((0, 3), dtype=np.int32), "n_triangles"),
])
def test_invalid_meshes_rejected(V, T, what):
    with pytest.raises(hm.HMError) as e:
        hm.hm_build(V, T, hm.hm_params_default(), stream=0)
    assert e.value.status == -1 and what in str(e.value)


def test_null_handle_calls():
    L = hm.lib()
    assert L.hm_matvec(None, None, None, 1, 1, 0, None) == -1
    assert L.hm_matvec_T(None, None, None, 1, 1, 0, None) == -1
    assert L.hm_solve(None, None, None, 1, 1, 0, None, None, None) == -1
    assert L.hm_query(None, 0, None, 0, None) == -1
    L.hm_free(None)           # NULL-safe
    assert "NULL" in hm.hm_last_error() or hm.hm_last_error() == ""


def test_null_build_out():
    L = hm.lib()
    assert L.hm_build(None, 3, None, 1, None, None, None) == -1


def _raw_batch(V, voff, T, toff, n_geom, p=None):
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    toff = np.ascontiguousarray(toff, dtype=np.int64)
    p = p or hm.hm_params_default()
    h = ctypes.c_void_p()
    st = hm.lib().hm_build_batch(V.ctypes.data, voff.ctypes.data, T.ctypes.data, toff.ctypes.data,
                                 n_geom, ctypes.byref(p), None, ctypes.byref(h))
    return st, h.value


@pytest.mark.parametrize("case,what", [
    ("n_geom0", "n_geom"), ("offsets", "start at 0"), ("empty", "no triangle"),
    ("local_index", "out of range"), ("degenerate_second", "geometry 1"),
])
def test_invalid_batches_rejected(case, what):
    V1, T1 = _tri()
    V = np.concatenate([V1, V1 + 5.0])
    T = np.concatenate([T1, T1])          # indices local to each mesh
    voff, toff, G = [0, 3, 6], [0, 1, 2], 2
    if case == "n_geom0":
        G = 0
    elif case == "offsets":
        toff = [1, 1, 2]
    elif case == "empty":
        toff = [0, 1, 1]
    elif case == "local_index":
        T = np.concatenate([T1, T1 + 3])  # global instead of local indices
    elif case == "degenerate_second":
        V = np.concatenate([V1, np.zeros((3, 3))])
    st, h = _raw_batch(V, voff, T, toff, G)
    assert st == -1 and h is None and what in hm.hm_last_error()


def test_null_build_batch_arguments():
    L = hm.lib()
    assert L.hm_build_batch(None, None, None, None, 1, None, None, None) == -1


class _FakeCuda:
    """Stands in for a device tensor in the binding's argument checks; its
    data pointer is never dereferenced because the checks fail first."""
    is_cuda = True

    def __init__(self, shape, dtype):
        import torch
        self.shape = tuple(shape)
        self.dtype = dtype
        self._t = torch.empty(0)

    def dim(self):
        return len(self.shape)

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return 4096


def test_wrong_length_rejected_before_any_device_access(monkeypatch):
    """A vector whose row count differs from the handle's is refused by the
    binding (HMatrix) and, for a raw handle, by the library itself."""
    import torch
    H = hm.HMatrix.__new__(hm.HMatrix)
    H.n, H._h = 1280, None
    x = _FakeCuda((1000,), torch.float64)
    with pytest.raises(hm.HMError) as e:
        H.matvec(x, out=_FakeCuda((1000,), torch.float64))
    assert e.value.status == hm.HM_ERR_ARG and "rows" in str(e.value)
    with pytest.raises(hm.HMError):
        H.solve(x)
    monkeypatch.setattr(torch, "Tensor", _FakeCuda)
    with pytest.raises(hm.HMError) as e:
        hm.hm_matvec(None, _FakeCuda((8, 2), torch.float64), _FakeCuda((8, 3), torch.float64))
    assert "same shape" in str(e.value)


def test_solve_refine_arguments_checked_in_header_order():
    """refine / inner_tol are part of the solve parameters, and their checks
    come after the handle check (a NULL handle is reported first)."""
    sp = hm.SolveParams(tol=1e-8, restart=10, max_iter=10, refine=1, inner_tol=2.0)
    L = hm.lib()
    assert L.hm_solve(None, None, None, 1, 1, 0, ctypes.byref(sp), None, None) == -1
    assert "NULL handle" in hm.hm_last_error()
