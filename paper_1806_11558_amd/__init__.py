"""MI355X (gfx950) H-matrix library for the Laplace single-layer BIE.

Python binding of ``libhm.so`` (C ABI in ``include/hm.h``).  The binding only
marshals arguments: every step of the setup, the products and the solve runs
in the library's HIP kernels.  If the library is not built, every call raises
``HMLibraryMissing``; there is no fallback.
"""
from ._binding import (  # noqa: F401
    HM_AUTOTUNE, HM_F32, HM_F32_F16, HM_F64, HM_GALERKIN, HM_OK, HM_NOT_CONVERGED, HM_PROFILE,
    HM_SOLVE_CG, HM_SOLVE_GRAPH, HM_STRICT, HM_ERR_ARG, HM_ERR_OOM, HM_ERR_HIP, HM_ERR_ACA, HM_ERR_STATE,
    ACA_CLASSES, HMError, HMLibraryMissing, HMatrix, Params, SolveInfo, SolveParams, Stats,
    hm_build, hm_build_batch, hm_entries, hm_free, hm_last_error, hm_matvec, hm_matvec_T,
    hm_params_default, hm_query, hm_solve, hm_solve_noalloc, lib, library_path, release_memory,
)


def __getattr__(name):
    # the differentiable solve needs torch; import it on first use
    if name in ("HSolve", "hsolve"):
        from . import adjoint
        return getattr(adjoint, name)
    raise AttributeError(name)
