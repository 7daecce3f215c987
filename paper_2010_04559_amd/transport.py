"""Python face of the HIP transport library: a handle per problem, torch
tensors for device memory and the current HIP stream for ordering.

Every operation runs in the library's HIP kernels; this module only
marshals arguments.
"""
import ctypes

import numpy as np

from . import _lib
from .inputs import Problem

_MODES = {"f64": _lib.TR_PREC_F64, "mixed": _lib.TR_PREC_MIXED, "sg": _lib.TR_PREC_SG,
          "mixed_bf16": _lib.TR_PREC_MIXED_BF16}
_ZSTORE = {"auto": _lib.TR_Z_AUTO, "keep": _lib.TR_Z_KEEP, "recompute": _lib.TR_Z_RECOMPUTE}


def problem_struct(prob: Problem):
    """The tr_problem of a problem description, with the host arrays it
    points to (keep the second value alive while the struct is used)."""
    p = _lib.TrProblem()
    p.dim = prob.dim
    for d in range(3):
        p.n[d] = int(prob.n[d]) if d < len(prob.n) else 1
        p.len[d] = float(prob.length[d])
    a = prob.angular
    p.ang_base_level = a.base_level
    for d in range(3):
        p.cone_axis[d] = float(a.cone_axis[d])
    p.cone_half_angle_deg = float(a.cone_half_angle_deg)
    p.cone_extra_levels = int(a.extra_levels)
    p.irregularity_closure = 1 if a.closure else 0
    p.band_lmax = int(a.band_lmax)
    bases = {"lin": _lib.TR_BASIS_LIN, "const": _lib.TR_BASIS_CONST}
    if a.basis not in bases:
        raise ValueError("angular basis is 'lin' or 'const'")
    p.angular_basis = bases[a.basis]
    st = np.ascontiguousarray(prob.sigma_t, dtype=np.float64)
    ss = np.ascontiguousarray(prob.sigma_s, dtype=np.float64)
    mom = np.ascontiguousarray(prob.moments(max([prob.order] + list(prob.mg_orders))), dtype=np.float64)
    order = np.ascontiguousarray(prob.mg_orders, dtype=np.int32)
    p.sigma_t = st.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.sigma_s = ss.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.order = prob.order
    p.moments = mom.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.n_levels = len(prob.mg_orders)
    p.mg_order = order.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    p.nu_pre, p.nu_post, p.nu_coarse = prob.nu_pre, prob.nu_post, prob.nu_coarse
    p.nu_post_coarse = prob.nu_post_coarse
    if sorted(prob.octant_order) != list(range(8)):
        raise ValueError("octant_order must be a permutation of 0..7")
    for i in range(8):
        p.octant_order[i] = int(prob.octant_order[i])
    return p, (st, ss, mom, order)


def solve_opts(prob: Problem, tol=None, restart=None, max_restarts=200, mode="f64", timing=False, z_store="auto"):
    o = _lib.TrSolveOpts()
    o.tol = prob.tol if tol is None else tol
    o.restart = prob.restart if restart is None else restart
    o.max_restarts = max_restarts
    o.prec_mode = _MODES[mode]
    o.timing = 1 if timing else 0
    o.z_store = _ZSTORE[z_store]
    return o


def workspace_bytes(prob: Problem, mode=None, restart=None, z_store="auto"):
    """Device bytes a handle for ``prob`` holds after setup (mode None), or
    after a solve in that preconditioner mode (host computation only)."""
    lib = _lib.load()
    p, keep = problem_struct(prob)
    o = solve_opts(prob, restart=restart, mode=mode, z_store=z_store) if mode is not None else None
    out = ctypes.c_size_t()
    _lib.check(lib.tr_workspace_bytes(ctypes.byref(p), ctypes.byref(o) if o is not None else None,
                                      ctypes.byref(out)))
    return out.value


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Transport:
    """One discretised problem on the current HIP device."""

    def __init__(self, prob: Problem):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.lib = _lib.load()
        self.prob = prob
        p, self._host_arrays = problem_struct(prob)
        h = ctypes.c_void_p()
        _lib.check(self.lib.tr_setup(ctypes.byref(p), ctypes.byref(h)))
        self.h = h
        info = _lib.TrInfo()
        _lib.check(self.lib.tr_info(self.h, ctypes.byref(info)))
        self.info = info
        self.C = info.cells
        self.S = info.spatial_dofs
        self.patches = [info.patches[l] for l in range(info.n_levels)]
        self.nlev = info.n_levels
        # scatter form per level: ("dense" | "factored" | "octant", R or K)
        names = {_lib.TR_SCATTER_DENSE: "dense", _lib.TR_SCATTER_FACTORED: "factored",
                 _lib.TR_SCATTER_OCTANT: "octant"}
        self.scatter_forms = [(names[info.scatter_form[l]], info.scatter_axes[l] or info.scatter_k[l])
                              for l in range(info.n_levels)]
        self.outer_axes = info.outer_axes
        self.sweep_lds = {"f64": bool(info.sweep_lds[0]), "f32": bool(info.sweep_lds[1])}
        self.sweep_pair = {"f64": bool(info.sweep_pair[0]), "f32": bool(info.sweep_pair[1])}
        self.dev = torch.device("cuda")

    def close(self):
        if getattr(self, "h", None):
            self.lib.tr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self):
        """Device memory the handle holds now (setup plus solver workspace)."""
        info = _lib.TrInfo()
        _lib.check(self.lib.tr_info(self.h, ctypes.byref(info)))
        return info.device_bytes

    # ------------------------------------------------------------ sizes
    def n(self, level=None):
        level = self.nlev - 1 if level is None else level
        return 3 * self.patches[level] * self.S

    def zeros(self, level=None, dtype=None):
        torch = _torch()
        return torch.zeros(self.n(level), dtype=dtype or torch.float64, device=self.dev)

    # ------------------------------------------------------------ data
    def rhs(self):
        torch = _torch()
        prob = self.prob
        b = self.zeros()
        q = torch.as_tensor(np.asarray(prob.q_cell, dtype=np.float64), device=self.dev)
        inf = None
        if prob.inflow is not None:
            f = prob.inflow
            inf = _lib.TrInflow()
            inf.kind = _lib.TR_INFLOW_ISO if f.kind == "iso" else _lib.TR_INFLOW_BEAM
            inf.axis, inf.side = f.axis, f.side
            for d in range(3):
                inf.lo[d] = int(min(f.lo[d], 2 ** 30))
                inf.hi[d] = int(min(f.hi[d], 2 ** 30))
                inf.direction[d] = float(f.direction[d])
            inf.value = float(f.value)
        _lib.check(self.lib.tr_rhs(self.h, _ptr(q), ctypes.byref(inf) if inf is not None else None, _ptr(b),
                                   _stream()))
        return b

    def detector(self, lo=None, hi=None):
        if lo is None:
            lo, hi = self.prob.detector
        w = self.zeros()
        lo_a = (ctypes.c_int * 3)(*[int(v) for v in lo])
        hi_a = (ctypes.c_int * 3)(*[int(v) for v in hi])
        _lib.check(self.lib.tr_detector(self.h, lo_a, hi_a, _ptr(w), _stream()))
        return w

    def response(self, w, phi):
        """R = w . phi (the detector response) formed by the library."""
        R = ctypes.c_double()
        _lib.check(self.lib.tr_response(self.h, _ptr(w), _ptr(phi), ctypes.byref(R), _stream()))
        return R.value

    def set_sigma(self, sigma_t, sigma_s):
        torch = _torch()
        st = torch.as_tensor(sigma_t, dtype=torch.float64, device=self.dev).contiguous()
        ss = torch.as_tensor(sigma_s, dtype=torch.float64, device=self.dev).contiguous()
        _lib.check(self.lib.tr_set_sigma(self.h, _ptr(st), _ptr(ss), _stream()))
        torch.cuda.current_stream().synchronize()

    # ------------------------------------------------------------ operators
    def _prec(self, t):
        torch = _torch()
        return _lib.TR_F64 if t.dtype == torch.float64 else _lib.TR_F32

    def sweep(self, level, g, adjoint=False):
        out = _torch().empty_like(g)
        fn = self.lib.tr_sweep_adjoint if adjoint else self.lib.tr_sweep
        _lib.check(fn(self.h, level, self._prec(g), _ptr(g), _ptr(out), _stream()))
        return out

    def scatter(self, level, phi, outer=False, split_bf16=False):
        """split_bf16: FP32 buffers, product from split-BF16 operands."""
        out = _torch().empty_like(phi)
        prec = _lib.TR_F32_SPLIT if split_bf16 else self._prec(phi)
        _lib.check(self.lib.tr_scatter(self.h, level, 1 if outer else 0, prec, _ptr(phi), _ptr(out), _stream()))
        return out

    def apply(self, x):
        y = _torch().empty_like(x)
        _lib.check(self.lib.tr_apply(self.h, _ptr(x), _ptr(y), _stream()))
        return y

    def prolong(self, level, xc):
        torch = _torch()
        out = torch.empty(self.n(level), dtype=xc.dtype, device=self.dev)
        _lib.check(self.lib.tr_transfer(self.h, level, _lib.TR_PROLONG, self._prec(xc), _ptr(xc), _ptr(out),
                                        _stream()))
        return out

    def restrict(self, level, xf):
        torch = _torch()
        out = torch.empty(self.n(level - 1), dtype=xf.dtype, device=self.dev)
        _lib.check(self.lib.tr_transfer(self.h, level, _lib.TR_RESTRICT, self._prec(xf), _ptr(xf), _ptr(out),
                                        _stream()))
        return out

    def coarse_gs(self, f, nu, adjoint=False):
        out = _torch().empty_like(f)
        _lib.check(self.lib.tr_coarse_gs(self.h, nu, 1 if adjoint else 0, _ptr(f), _ptr(out), _stream()))
        return out

    def vcycle(self, r, mode="f64", adjoint=False):
        z = _torch().empty_like(r)
        _lib.check(self.lib.tr_mg_vcycle(self.h, _MODES[mode], 1 if adjoint else 0, _ptr(r), _ptr(z), _stream()))
        return z

    def _opts(self, tol, restart, max_restarts, mode, timing, z_store="auto"):
        return solve_opts(self.prob, tol, restart, max_restarts, mode, timing, z_store)

    def solve(self, b, tol=None, restart=None, max_restarts=200, mode="f64", timing=False, check=True,
              z_store="auto", method="gmres"):
        """GMRES(restart) (method "gmres") or BiCGStab ("bicgstab", at most
        restart x (max_restarts + 1) iterations)."""
        x = _torch().empty_like(b)
        o = self._opts(tol, restart, max_restarts, mode, timing, z_store)
        st = _lib.TrSolveStats()
        fn = {"gmres": self.lib.tr_gmres_solve, "bicgstab": self.lib.tr_bicgstab_solve}[method]
        rc = fn(self.h, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(st), _stream())
        _lib.check(rc, allow=() if check else (_lib.TR_ERR_NOCONV,))
        return x, st.as_dict()

    def adjoint_grad(self, w, phi, tol=None, restart=None, max_restarts=200, mode="f64", timing=False):
        torch = _torch()
        lam = torch.empty_like(phi)
        gt = torch.empty(self.C, dtype=torch.float64, device=self.dev)
        gs = torch.empty(self.C, dtype=torch.float64, device=self.dev)
        o = self._opts(tol, restart, max_restarts, mode, timing)
        st = _lib.TrSolveStats()
        _lib.check(self.lib.tr_adjoint_grad(self.h, _ptr(w), _ptr(phi), _ptr(lam), _ptr(gt), _ptr(gs),
                                            ctypes.byref(o), ctypes.byref(st), _stream()))
        return gt, gs, lam, st.as_dict()

    def time_sweep_kernel(self, level=None, prec="f64", reps=10):
        level = self.nlev - 1 if level is None else level
        ms = ctypes.c_double()
        _lib.check(self.lib.tr_time_sweep_kernel(self.h, level, _lib.TR_F64 if prec == "f64" else _lib.TR_F32,
                                                 reps, ctypes.byref(ms), _stream()))
        return ms.value

    def sweep_kernel_name(self, level=None, prec="f64"):
        """Name of the forward-sweep kernel the library launches."""
        t = "double" if prec == "f64" else "float"
        if self.sweep_pair[prec]:
            return "k_sweep_pair<%s>" % t
        return ("k_sweep_lds<%s,%d>" if self.sweep_lds[prec] else "k_sweep<%s,%d>") % (t, self.prob.dim)

    def scatter_flops(self, level=None, outer=False):
        """Multiply-add flops per application of a level's scatter product as
        the library forms it (the problem operator's with outer)."""
        level = self.nlev - 1 if level is None else level
        A, S = 3 * self.patches[level], self.S
        if outer:
            return 2.0 * A * A * S / 2 ** self.outer_axes
        form, k = self.scatter_forms[level]
        if form == "octant":
            return 2.0 * A * A * S / 2 ** k
        if form == "factored":
            return 4.0 * A * k * S
        return 2.0 * A * A * S

    def time_scatter_kernel(self, level=None, outer=False, prec="f64", reps=10):
        level = self.nlev - 1 if level is None else level
        ms = ctypes.c_double()
        code = {"f64": _lib.TR_F64, "f32": _lib.TR_F32, "bf16x3": _lib.TR_F32_SPLIT}[prec]
        _lib.check(self.lib.tr_time_scatter_kernel(self.h, level, 1 if outer else 0, code, reps,
                                                   ctypes.byref(ms), _stream()))
        return ms.value
