"""ctypes declarations of the C ABI in include/tr.h (argument marshalling only).

The shared library is paper_2010_04559_amd/libtr.so, built in-tree by
``paper_2010_04559_amd.build.build()``.  Loading fails loudly when it is
missing: there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtr.so")

TR_OK, TR_ERR_ARG, TR_ERR_UNSUPPORTED, TR_ERR_ALLOC, TR_ERR_HIP, TR_ERR_NOCONV = range(6)
TR_F64, TR_F32, TR_F32_SPLIT = 0, 1, 2
TR_PREC_F64, TR_PREC_MIXED, TR_PREC_SG, TR_PREC_MIXED_BF16 = 0, 1, 2, 3
TR_INFLOW_NONE, TR_INFLOW_ISO, TR_INFLOW_BEAM = 0, 1, 2
TR_RESTRICT, TR_PROLONG = 0, 1
TR_Z_AUTO, TR_Z_KEEP, TR_Z_RECOMPUTE = 0, 1, 2
TR_SCATTER_DENSE, TR_SCATTER_FACTORED, TR_SCATTER_OCTANT = 0, 1, 2
TR_BASIS_LIN, TR_BASIS_CONST = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class TrProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("len", ctypes.c_double * 3),
                ("ang_base_level", ctypes.c_int), ("cone_axis", ctypes.c_double * 3),
                ("cone_half_angle_deg", ctypes.c_double), ("cone_extra_levels", ctypes.c_int),
                ("irregularity_closure", ctypes.c_int), ("band_lmax", ctypes.c_int), ("sigma_t", _dp), ("sigma_s", _dp),
                ("order", ctypes.c_int), ("moments", _dp), ("n_levels", ctypes.c_int),
                ("mg_order", _ip), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("nu_coarse", ctypes.c_int), ("octant_order", ctypes.c_int * 8), ("angular_basis", ctypes.c_int),
                ("nu_post_coarse", ctypes.c_int)]


class TrInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("cells", ctypes.c_int), ("spatial_dofs", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("patches", ctypes.c_int * 16), ("order_outer", ctypes.c_int),
                ("device_bytes", ctypes.c_size_t), ("scatter_form", ctypes.c_int * 16),
                ("scatter_axes", ctypes.c_int * 16), ("scatter_k", ctypes.c_int * 16), ("outer_axes", ctypes.c_int),
                ("sweep_lds", ctypes.c_int * 2), ("sweep_pair", ctypes.c_int * 2)]


class TrInflow(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("axis", ctypes.c_int), ("side", ctypes.c_int),
                ("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3), ("value", ctypes.c_double),
                ("direction", ctypes.c_double * 3)]


class TrSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("prec_mode", ctypes.c_int), ("timing", ctypes.c_int), ("z_store", ctypes.c_int)]


class TrSolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("ms_total", ctypes.c_double), ("ms_sweep", ctypes.c_double),
                ("ms_scatter", ctypes.c_double), ("ms_transfer", ctypes.c_double),
                ("ms_coarse", ctypes.c_double), ("ms_apply", ctypes.c_double), ("ms_orth", ctypes.c_double),
                ("ms_other", ctypes.c_double), ("n_sweep", ctypes.c_int), ("n_scatter", ctypes.c_int),
                ("n_coarse", ctypes.c_int), ("ms_sweep_finest", ctypes.c_double),
                ("n_sweep_finest", ctypes.c_int), ("n_precond", ctypes.c_int),
                ("sweep_dof_updates", ctypes.c_double), ("coarse_steps", ctypes.c_int),
                ("flexible", ctypes.c_int), ("ms_scatter_outer", ctypes.c_double), ("n_scatter_outer", ctypes.c_int),
                ("ms_scatter_finest", ctypes.c_double), ("n_scatter_finest", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_vp = ctypes.c_void_p
_h = ctypes.c_void_p
SIGNATURES = {
    "tr_setup": (ctypes.c_int, [ctypes.POINTER(TrProblem), ctypes.POINTER(_h)]),
    "tr_destroy": (None, [_h]),
    "tr_last_error": (ctypes.c_char_p, []),
    "tr_info": (ctypes.c_int, [_h, ctypes.POINTER(TrInfo)]),
    "tr_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(TrProblem), ctypes.POINTER(TrSolveOpts),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "tr_set_sigma": (ctypes.c_int, [_h, _vp, _vp, _vp]),
    "tr_response": (ctypes.c_int, [_h, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]),
    "tr_rhs": (ctypes.c_int, [_h, _vp, ctypes.POINTER(TrInflow), _vp, _vp]),
    "tr_detector": (ctypes.c_int, [_h, _ip, _ip, _vp, _vp]),
    "tr_sweep": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_sweep_adjoint": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_scatter": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_apply": (ctypes.c_int, [_h, _vp, _vp, _vp]),
    "tr_transfer": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_coarse_gs": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_coarse_gs_noalloc": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_mg_vcycle": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "tr_gmres_solve": (ctypes.c_int, [_h, _vp, _vp, ctypes.POINTER(TrSolveOpts), ctypes.POINTER(TrSolveStats), _vp]),
    "tr_bicgstab_solve": (ctypes.c_int, [_h, _vp, _vp, ctypes.POINTER(TrSolveOpts), ctypes.POINTER(TrSolveStats),
                                         _vp]),
    "tr_adjoint_grad": (ctypes.c_int, [_h, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(TrSolveOpts),
                                       ctypes.POINTER(TrSolveStats), _vp]),
    "tr_time_sweep_kernel": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_double), _vp]),
    "tr_time_scatter_kernel": (ctypes.c_int, [_h, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_double), _vp]),
}

_lib = None


class TrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tr error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libtr.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing: run paper_2010_04559_amd.build.build() first" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc, allow=()):
    if rc != TR_OK and rc not in allow:
        raise TrError(rc, load().tr_last_error().decode())
    return rc
