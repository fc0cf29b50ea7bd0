"""ctypes binding of libhm.so: the C calls under their own names plus a small
``HMatrix`` convenience class.  Device vectors are torch tensors (memory and
streams only); the binding never computes anything itself."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HM_OK, HM_NOT_CONVERGED = 0, 1
HM_ERR_ARG, HM_ERR_OOM, HM_ERR_HIP, HM_ERR_ACA, HM_ERR_STATE = -1, -2, -3, -4, -5
HM_F64, HM_F32, HM_F32_F16 = 0, 1, 2
HM_SOLVE_GRAPH = 1
HM_SOLVE_CG = 2
HM_AUTOTUNE = 4
HM_STRICT = 1
HM_PROFILE = 2
HM_GALERKIN = 8
(HM_Q_STATS, HM_Q_MORTON, HM_Q_PERM, HM_Q_CLUSTERS, HM_Q_BOXES, HM_Q_DENSE_BLOCKS,
 HM_Q_LR_BLOCKS, HM_Q_LEAVES, HM_Q_TIMINGS, HM_Q_LR_FACTORS, HM_Q_KERNEL_TIMES,
 HM_Q_TUNE, HM_Q_DENSE_ENTRIES, HM_Q_ACA_BINS, HM_Q_ACA_TUNE) = range(15)
ACA_CLASSES = ("wg1024", "wg256", "wave4", "wave2", "wave1", "wg128")
HM_NPHASE = 8
HM_NKERNEL = 8
KERNELS = ("fwd_gather", "fwd_vtx", "fwd_unused", "fwd_panels",
           "tr_gather", "tr_panel_dots", "tr_block_sums", "tr_columns")
PHASES = ("geometry", "morton_sort", "tree_boxes", "partition", "near_field", "aca",
          "pack_items", "total")

_STATUS = {HM_ERR_ARG: "HM_ERR_ARG", HM_ERR_OOM: "HM_ERR_OOM", HM_ERR_HIP: "HM_ERR_HIP",
           HM_ERR_ACA: "HM_ERR_ACA", HM_ERR_STATE: "HM_ERR_STATE"}


class HMLibraryMissing(RuntimeError):
    pass


class HMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("max_rank", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_int32), ("eta", C.c_double), ("aca_eps", C.c_double),
                ("mem_limit_bytes", C.c_int64)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("transpose", C.c_int32), ("use_x0", C.c_int32), ("flags", C.c_int32),
                ("refine", C.c_int32), ("inner_tol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("ir_steps", C.c_int32), ("rel_residual", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n", "n_clusters", "n_leaves", "n_dense", "n_lr", "depth", "dense_entries",
        "lr_entries", "lr_u_entries", "stored_bytes", "rank_sum", "rank_max", "cap_hits", "aca_entry_evals",
        "n_panel_cols", "n_titems", "device_bytes", "precision", "aca_chunks", "n_geom",
        "unit_cols")]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def library_path() -> str:
    return os.environ.get("HM_LIBRARY", os.path.join(_HERE, "libhm.so"))


def lib():
    """Load libhm.so (raises HMLibraryMissing if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise HMLibraryMissing(
            f"{path} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    try:
        # load torch's HIP runtime first, so that the library and torch share
        # one runtime (same soname) and device pointers move freely between them
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hm_params_default.argtypes = [C.POINTER(Params)]
    L.hm_build.argtypes = [vp, i64, vp, i64, C.POINTER(Params), vp, C.POINTER(vp)]
    L.hm_build_batch.argtypes = [vp, vp, vp, vp, i32, C.POINTER(Params), vp, C.POINTER(vp)]
    L.hm_matvec.argtypes = [vp, vp, vp, i64, i32, i32, vp]
    L.hm_matvec_T.argtypes = [vp, vp, vp, i64, i32, i32, vp]
    L.hm_solve.argtypes = [vp, vp, vp, i64, i32, i32, C.POINTER(SolveParams),
                           C.POINTER(SolveInfo), vp]
    L.hm_solve_noalloc.argtypes = L.hm_solve.argtypes
    L.hm_free.argtypes = [vp]
    L.hm_free.restype = None
    L.hm_query.argtypes = [vp, i32, vp, i64, C.POINTER(i64)]
    L.hm_entries.argtypes = [vp, vp, vp, i64, vp]
    L.hm_last_error.restype = C.c_char_p
    L.hm_last_error.argtypes = []
    L.hm_release_memory.argtypes = []
    for f in ("hm_params_default", "hm_build", "hm_build_batch", "hm_release_memory", "hm_matvec", "hm_matvec_T", "hm_solve",
              "hm_solve_noalloc", "hm_query", "hm_entries"):
        getattr(L, f).restype = C.c_int
    _LIB = L
    return L


def hm_last_error() -> str:
    return lib().hm_last_error().decode()


def _check(status: int, ok=(HM_OK,)) -> int:
    if status not in ok:
        raise HMError(status, hm_last_error())
    return status


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ---------------------------------------------------------------- C calls

def hm_params_default() -> Params:
    p = Params()
    _check(lib().hm_params_default(C.byref(p)))
    return p


def hm_build(vertices: np.ndarray, triangles: np.ndarray, params: Params, stream=None) -> int:
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(triangles, dtype=np.int32)
    if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
        raise HMError(HM_ERR_ARG, "vertices and triangles must be [*, 3]")
    h = C.c_void_p()
    _check(lib().hm_build(v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0], C.byref(params),
                          _stream_ptr(stream), C.byref(h)))
    return h.value


def release_memory() -> None:
    """Return the device memory cached in the library's pool (freed handles,
    build temporaries) to the device (hm_release_memory)."""
    _check(lib().hm_release_memory())


def hm_build_batch(meshes, params: Params, stream=None) -> int:
    """meshes: sequence of (vertices [nv, 3], triangles [nt, 3]) with indices
    local to each mesh."""
    vs = [np.ascontiguousarray(v, dtype=np.float64) for v, _ in meshes]
    ts = [np.ascontiguousarray(t, dtype=np.int32) for _, t in meshes]
    for v, t in zip(vs, ts):
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise HMError(HM_ERR_ARG, "vertices and triangles must be [*, 3]")
    voff = np.concatenate([[0], np.cumsum([v.shape[0] for v in vs])]).astype(np.int64)
    toff = np.concatenate([[0], np.cumsum([t.shape[0] for t in ts])]).astype(np.int64)
    V = np.ascontiguousarray(np.concatenate(vs))
    T = np.ascontiguousarray(np.concatenate(ts))
    h = C.c_void_p()
    _check(lib().hm_build_batch(V.ctypes.data, voff.ctypes.data, T.ctypes.data, toff.ctypes.data,
                                len(meshes), C.byref(params), _stream_ptr(stream), C.byref(h)))
    return h.value


def _vec_args(x):
    """(rows, nrhs, dtype code) of a device vector [n] or [n, nrhs]."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise HMError(HM_ERR_ARG, "vectors must be CUDA tensors")
    if x.dtype not in (torch.float32, torch.float64):
        raise HMError(HM_ERR_ARG, "vectors must be float32 or float64")
    if not x.is_contiguous():
        raise HMError(HM_ERR_ARG, "vectors must be contiguous")
    if x.dim() not in (1, 2):
        raise HMError(HM_ERR_ARG, f"vector shape {tuple(x.shape)}: expected [n] or [n, nrhs]")
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    return x.shape[0], nrhs, (HM_F32 if x.dtype == torch.float32 else HM_F64)


def _pair_args(a, b, what):
    na, nrhs, dt = _vec_args(a)
    if a.shape != b.shape or a.dtype != b.dtype:
        raise HMError(HM_ERR_ARG, f"{what} must have the same shape and dtype")
    _vec_args(b)
    return na, nrhs, dt


def hm_matvec(h: int, x, y, stream=None, transpose: bool = False) -> None:
    """y = H x (or H^T x).  The library checks the row count against the
    handle's number of unknowns."""
    n, nrhs, dt = _pair_args(x, y, "x and y")
    f = lib().hm_matvec_T if transpose else lib().hm_matvec
    _check(f(h, x.data_ptr(), y.data_ptr(), n, nrhs, dt, _stream_ptr(stream)))


def hm_matvec_T(h: int, x, y, stream=None) -> None:
    hm_matvec(h, x, y, stream, transpose=True)


def hm_solve(h: int, f, sigma, sp: SolveParams, stream=None) -> tuple[int, SolveInfo]:
    n, nrhs, dt = _pair_args(f, sigma, "f and sigma")
    info = SolveInfo()
    st = lib().hm_solve(h, f.data_ptr(), sigma.data_ptr(), n, nrhs, dt, C.byref(sp),
                        C.byref(info), _stream_ptr(stream))
    _check(st, ok=(HM_OK, HM_NOT_CONVERGED))
    return st, info


def hm_solve_noalloc(h: int, f, sigma, sp: SolveParams, stream=None) -> tuple[int, SolveInfo]:
    """hm_solve with its workspace in the library's fixed device array (no
    allocation; HM_NOALLOC_SCRATCH_BYTES at most)."""
    n, nrhs, dt = _pair_args(f, sigma, "f and sigma")
    info = SolveInfo()
    st = lib().hm_solve_noalloc(h, f.data_ptr(), sigma.data_ptr(), n, nrhs, dt, C.byref(sp),
                                C.byref(info), _stream_ptr(stream))
    _check(st, ok=(HM_OK, HM_NOT_CONVERGED))
    return st, info


def hm_free(h: int) -> None:
    if h:
        lib().hm_free(h)


def hm_query(h: int, what: int, dst: np.ndarray | None = None) -> np.ndarray | int:
    need = C.c_int64(0)
    if dst is None:
        lib().hm_query(h, what, None, 0, C.byref(need))
        return int(need.value)
    _check(lib().hm_query(h, what, dst.ctypes.data, dst.nbytes, C.byref(need)))
    return dst


def hm_entries(h: int, rows, cols) -> np.ndarray:
    r = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1)
    c = np.ascontiguousarray(cols, dtype=np.int32).reshape(-1)
    if r.shape != c.shape:
        raise HMError(HM_ERR_ARG, "rows and cols differ in length")
    out = np.empty(r.size, dtype=np.float64)
    _check(lib().hm_entries(h, r.ctypes.data, c.ctypes.data, r.size, out.ctypes.data))
    return out


# ---------------------------------------------------------------- convenience

class HMatrix:
    """An H-matrix built on the current CUDA device (see include/hm.h)."""

    def __init__(self, vertices, triangles, *, leaf_size: int = 32, eta: float = 1.0,
                 eps: float = 1e-6, max_rank: int = 64, precision: str = "f64",
                 strict: bool = False, profile: bool = False, mem_limit_bytes: int = 0,
                 autotune: bool = False, operator: str = "collocation", stream=None):
        """operator: "collocation" (centroid collocation) or "galerkin"
        (HM_GALERKIN: the Galerkin matrix with piecewise constants)."""
        p = self._params(leaf_size, eta, eps, max_rank, precision, strict, profile,
                         mem_limit_bytes, autotune, operator)
        self.n = int(np.asarray(triangles).shape[0])
        self.offsets = np.array([0, self.n], dtype=np.int64)
        self._h = hm_build(vertices, triangles, p, stream)

    @classmethod
    def batch(cls, meshes, *, leaf_size: int = 32, eta: float = 1.0, eps: float = 1e-6,
              max_rank: int = 64, precision: str = "f64", strict: bool = False,
              profile: bool = False, mem_limit_bytes: int = 0, autotune: bool = False,
              operator: str = "collocation", stream=None):
        """One handle for several meshes [(vertices, triangles), ...]
        (hm_build_batch); unknowns are the triangles in concatenated order."""
        self = cls.__new__(cls)
        p = self._params(leaf_size, eta, eps, max_rank, precision, strict, profile,
                         mem_limit_bytes, autotune, operator)
        sizes = [int(np.asarray(t).shape[0]) for _, t in meshes]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self._h = hm_build_batch(meshes, p, stream)
        return self

    def _params(self, leaf_size, eta, eps, max_rank, precision, strict, profile, mem_limit_bytes,
                autotune=False, operator="collocation"):
        if operator not in ("collocation", "galerkin"):
            raise HMError(HM_ERR_ARG, f"unknown operator {operator!r}")
        p = hm_params_default()
        p.leaf_size = leaf_size
        p.eta = eta
        p.aca_eps = eps
        p.max_rank = max_rank
        p.precision = {"f64": HM_F64, "f32": HM_F32, "f16": HM_F32_F16}[precision]
        p.flags = ((HM_STRICT if strict else 0) | (HM_PROFILE if profile else 0)
                   | (HM_AUTOTUNE if autotune else 0)
                   | (HM_GALERKIN if operator == "galerkin" else 0))
        self.operator = operator
        p.mem_limit_bytes = mem_limit_bytes
        self.params = p
        self.storage_dtype = np.float64 if precision == "f64" else np.float32
        self._h = None
        return p

    # products -------------------------------------------------------------
    def _rows(self, v):
        if getattr(v, "shape", (None,))[0] != self.n:
            raise HMError(HM_ERR_ARG, f"vector has {v.shape[0]} rows, the H-matrix {self.n}")

    def matvec(self, x, out=None, stream=None, transpose: bool = False):
        import torch
        self._rows(x)
        y = torch.empty_like(x) if out is None else out
        self._rows(y)
        hm_matvec(self._h, x, y, stream, transpose)
        return y

    def matvec_T(self, x, out=None, stream=None):
        return self.matvec(x, out, stream, transpose=True)

    def solve(self, f, *, tol: float = 1e-8, restart: int = 100, max_iter: int = 1000,
              transpose: bool = False, x0=None, graph: bool = False, refine: bool = False,
              inner_tol: float = 0.0, method: str = "gmres", stream=None):
        """GMRES on H s = f (hm_solve); with refine=True iterative refinement
        around an inner GMRES with float products to inner_tol; method="cg"
        for conjugate gradients (HM_SOLVE_CG, the Galerkin system).  Returns
        (sigma, info, status); status HM_NOT_CONVERGED is returned, not
        raised."""
        if method not in ("gmres", "cg"):
            raise HMError(HM_ERR_ARG, f"unknown method {method!r}")
        import torch
        self._rows(f)
        sp = SolveParams(tol=tol, restart=restart, max_iter=max_iter,
                         transpose=1 if transpose else 0, use_x0=0 if x0 is None else 1,
                         flags=(HM_SOLVE_GRAPH if graph else 0)
                         | (HM_SOLVE_CG if method == "cg" else 0),
                         refine=1 if refine else 0,
                         inner_tol=inner_tol)
        sigma = torch.empty_like(f) if x0 is None else x0.clone()
        st, info = hm_solve(self._h, f, sigma, sp, stream)
        return sigma, info, st

    # introspection --------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        _check(lib().hm_query(self._h, HM_Q_STATS, C.addressof(s), C.sizeof(s), None))
        return s.as_dict()

    def timings(self) -> dict:
        t = np.zeros(HM_NPHASE, dtype=np.float64)
        hm_query(self._h, HM_Q_TIMINGS, t)
        return dict(zip(PHASES, t.tolist()))

    def tune_results(self) -> np.ndarray:
        """[k, 2] (unit columns, ms per one-column product) timed by the
        autotuner (empty without autotune=True)."""
        need = hm_query(self._h, HM_Q_TUNE)
        out = np.zeros(need // 8, dtype=np.float64)
        if need:
            hm_query(self._h, HM_Q_TUNE, out)
        return out.reshape(-1, 2)

    def aca_bins(self) -> np.ndarray:
        """int32[8][2]: (largest max(m, n) of the size bin, ACA kernel class)
        the build ran with (classes in ACA_CLASSES order)."""
        return hm_query(self._h, HM_Q_ACA_BINS, np.zeros((8, 2), dtype=np.int32))

    def aca_tune(self) -> np.ndarray:
        """double[k][4] (bin, class, sampled blocks, ms) of every candidate the
        ACA binning tuner timed (empty without autotune)."""
        k = hm_query(self._h, HM_Q_ACA_TUNE) // 32
        if k == 0:
            return np.zeros((0, 4))
        return hm_query(self._h, HM_Q_ACA_TUNE, np.zeros((k, 4)))

    def kernel_times(self) -> dict:
        """Accumulated product-kernel milliseconds and launch counts since the
        last call (needs profile=True)."""
        t = np.zeros(2 * HM_NKERNEL, dtype=np.float64)
        hm_query(self._h, HM_Q_KERNEL_TIMES, t)
        return {k: {"ms": float(t[i]), "launches": int(t[HM_NKERNEL + i])}
                for i, k in enumerate(KERNELS)}

    def _q(self, what, dtype, cols):
        need = hm_query(self._h, what)
        out = np.empty(need // np.dtype(dtype).itemsize, dtype=dtype)
        hm_query(self._h, what, out)
        return out.reshape(-1, cols) if cols > 1 else out

    def morton_keys(self):
        return self._q(HM_Q_MORTON, np.uint64, 1)

    def perm(self):
        return self._q(HM_Q_PERM, np.int32, 1)

    def clusters(self):
        return self._q(HM_Q_CLUSTERS, np.int32, 4)

    def boxes(self):
        return self._q(HM_Q_BOXES, np.float64, 6)

    def leaves(self):
        return self._q(HM_Q_LEAVES, np.int32, 3)

    def dense_blocks(self):
        return self._q(HM_Q_DENSE_BLOCKS, np.int64, 6)

    def lr_blocks(self):
        return self._q(HM_Q_LR_BLOCKS, np.int64, 6)

    def lr_factors(self, b: int):
        """Plain U (m x r) and V (n x r) of low-rank block b."""
        blk = self.lr_blocks()[b]
        m, n, r = int(blk[1] - blk[0]), int(blk[3] - blk[2]), int(blk[4])
        size = np.dtype(self.storage_dtype).itemsize
        nbytes = r * (m + n) * size
        # the block index travels in the first 8 bytes of the buffer, which
        # holds at least those 8 bytes whatever the rank
        raw = np.zeros(max(nbytes, 8), dtype=np.uint8)
        raw[:8].view(np.int64)[0] = b
        _check(lib().hm_query(self._h, HM_Q_LR_FACTORS, raw.ctypes.data, raw.nbytes, None))
        buf = raw[:nbytes].view(self.storage_dtype)
        U = buf[: m * r].reshape(r, m).T.astype(np.float64)
        V = buf[m * r:].reshape(r, n).T.astype(np.float64)
        return U, V

    def dense_entries(self, b: int, blocks=None):
        """The stored entries of dense block b (in the order of
        dense_blocks(), which may be passed in), m x n, rows and columns in
        Morton order."""
        blk = (self.dense_blocks() if blocks is None else blocks)[b]
        m, n = int(blk[1] - blk[0]), int(blk[3] - blk[2])
        buf = np.zeros(max(m * n, 1), dtype=np.float64)
        buf.view(np.int64)[0] = b
        _check(lib().hm_query(self._h, HM_Q_DENSE_ENTRIES, buf.ctypes.data, buf.nbytes, None))
        return buf[: m * n].reshape(m, n)

    def entries(self, rows, cols):
        return hm_entries(self._h, rows, cols)

    def free(self):
        if getattr(self, "_h", None):
            hm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
