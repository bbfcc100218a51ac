"""Python binding of libshellconv (argument marshalling only).

Every computation runs in the HIP library; PyTorch only provides device memory and the
current stream.  The entry points mirror the C-ABI of include/shellconv.h:
plan create/destroy, layout, set_params, factor, step, newton_residual, set_base, jvp.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshellconv.so")

SC_FP64 = 0
SC_MIXED = 1
SC_MIXED_SOLVE_FP64 = 1   # mixed_solve of Plan
SC_MIXED_SOLVE_FP32 = 2
SC_CONT_RA = 0             # param of Continuation
SC_CONT_EK = 1
SC_CORIOLIS_IMPLICIT = 0   # coriolis of Plan
SC_CORIOLIS_EXPLICIT = 1
_ERRORS = {1: "SC_ERR_ARG", 2: "SC_ERR_STATE", 3: "SC_ERR_NONFINITE", 4: "SC_ERR_NOMEM",
           5: "SC_ERR_HIP", 6: "SC_ERR_INTERNAL"}


class ShellConvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("M", ctypes.c_int), ("m0", ctypes.c_int), ("N", ctypes.c_int),
                ("radius_ratio", ctypes.c_double), ("Ek", ctypes.c_double), ("Ra", ctypes.c_double),
                ("Pr", ctypes.c_double), ("dt", ctypes.c_double),
                ("nr_phys", ctypes.c_int), ("ntheta", ctypes.c_int), ("nphi", ctypes.c_int),
                ("device", ctypes.c_int), ("nvec_max", ctypes.c_int),
                ("refine_fp64", ctypes.c_int), ("refine_mixed", ctypes.c_int), ("mixed_solve", ctypes.c_int),
                ("coriolis", ctypes.c_int), ("graph_capture", ctypes.c_int)]


class _Layout(ctypes.Structure):
    _fields_ = [("n_real", ctypes.c_longlong), ("L", ctypes.c_int), ("M", ctypes.c_int), ("m0", ctypes.c_int),
                ("N", ctypes.c_int), ("K", ctypes.c_int), ("S", ctypes.c_int), ("Np", ctypes.c_int),
                ("ntheta", ctypes.c_int), ("nphi", ctypes.c_int), ("nvec_max", ctypes.c_int)]


class _NewtonOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("gmres_tol", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_newton", ctypes.c_int), ("max_matvec", ctypes.c_int), ("prec", ctypes.c_int),
                ("J", ctypes.c_longlong), ("forcing", ctypes.c_void_p)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("ring_fp32", ctypes.c_int), ("ring_fp64", ctypes.c_int), ("anal_folded", ctypes.c_int),
                ("ncand", ctypes.c_int), ("ms_fp32", ctypes.c_double), ("ms_fp64", ctypes.c_double),
                ("linear_mode", ctypes.c_int)]


class _ContOpts(ctypes.Structure):
    _fields_ = [("param", ctypes.c_int), ("n_opt", ctypes.c_int), ("gamma", ctypes.c_double),
                ("ra_coef", ctypes.c_double), ("refine_tol", ctypes.c_double), ("refine_growth", ctypes.c_double),
                ("max_retries", ctypes.c_int), ("newton", _NewtonOpts)]


class _ContPoint(ctypes.Structure):
    _fields_ = [("param", ctypes.c_double), ("Ra", ctypes.c_double), ("Ek", ctypes.c_double), ("C", ctypes.c_double),
                ("unorm", ctypes.c_double), ("cheb_ratio", ctypes.c_double), ("sh_ratio", ctypes.c_double),
                ("newton_steps", ctypes.c_int), ("matvecs", ctypes.c_int), ("converged", ctypes.c_int),
                ("state_mode", ctypes.c_int), ("refined", ctypes.c_int), ("retries", ctypes.c_int),
                ("L", ctypes.c_int), ("N", ctypes.c_int)]


class _NewtonReport(ctypes.Structure):
    _fields_ = [("newton_steps", ctypes.c_int), ("matvecs", ctypes.c_int), ("converged", ctypes.c_int),
                ("rnorm", ctypes.c_double * 65), ("step_matvecs", ctypes.c_int * 64), ("C", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2508_16635_amd.build`")
    # torch's HIP runtime must be the one in the process: loading the library first would bind
    # its libamdhip64 dependency to another copy and leave torch without a device
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "sc_plan_create": [ctypes.POINTER(vp), ctypes.POINTER(_Params)],
        "sc_plan_destroy": [vp],
        "sc_layout": [vp, ctypes.POINTER(_Layout)],
        "sc_set_params": [vp, d, d, d],
        "sc_factor": [vp, vp],
        "sc_step": [vp, vp, d, vp, vp],
        "sc_newton_residual": [vp, vp, d, vp, ctypes.POINTER(d), vp],
        "sc_newton_residual_noalloc": [vp, vp, d, vp, vp, vp],
        "sc_set_base": [vp, vp, d, ll, vp],
        "sc_jvp": [vp, i, vp, ll, vp, ll, i, vp],
        "sc_newton": [vp, vp, ctypes.POINTER(d), ctypes.POINTER(_NewtonOpts), ctypes.POINTER(_NewtonReport), vp],
        "sc_profile": [vp, i],
        "sc_profile_read": [vp, ctypes.POINTER(d), ctypes.POINTER(ll), i],
        "sc_autotune": [vp, i, i, ctypes.POINTER(_TuneReport), vp],
        "sc_set_kernels": [vp, i, i, i],
        "sc_get_kernels": [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)],
        "sc_batch_create": [ctypes.POINTER(vp), ctypes.POINTER(vp), i],
        "sc_batch_destroy": [vp],
        "sc_batch_jvp": [vp, ctypes.POINTER(i), ctypes.POINTER(vp), ctypes.POINTER(vp), i, vp],
        "sc_batch_newton": [vp, ctypes.POINTER(vp), ctypes.POINTER(d), ctypes.POINTER(_NewtonOpts),
                            ctypes.POINTER(_NewtonReport), vp],
        "sc_interpolate": [vp, vp, vp, vp, vp],
        "sc_tail_ratios": [vp, vp, ctypes.POINTER(d), ctypes.POINTER(d), vp],
        "sc_cont_create": [ctypes.POINTER(vp), vp, vp, d, ctypes.POINTER(_ContOpts), ctypes.POINTER(_ContPoint), vp],
        "sc_cont_step": [vp, d, ctypes.POINTER(_ContPoint), vp],
        "sc_cont_layout": [vp, ctypes.POINTER(_Layout)],
        "sc_cont_state": [vp, vp, ll, ctypes.POINTER(d), vp],
        "sc_cont_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sc_last_error.argtypes = []
    lib.sc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


STAGES = ["radial_prep", "legendre_synth", "ring", "legendre_anal", "project_rhs", "chain_solve",
          "T_solve", "residual64", "axpy", "finalize"]


def exported_symbols():
    return ["sc_plan_create", "sc_plan_destroy", "sc_layout", "sc_set_params", "sc_factor", "sc_step",
            "sc_newton_residual", "sc_set_base", "sc_jvp", "sc_newton", "sc_profile", "sc_profile_read",
            "sc_last_error", "sc_batch_create", "sc_batch_destroy", "sc_batch_jvp", "sc_autotune",
            "sc_batch_newton", "sc_newton_residual_noalloc", "sc_interpolate", "sc_tail_ratios",
            "sc_cont_create", "sc_cont_step", "sc_cont_layout", "sc_cont_state", "sc_cont_destroy",
            "sc_set_kernels", "sc_get_kernels"]


def _check(rc):
    if rc != 0:
        raise ShellConvError(rc, _lib.sc_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, n_min):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.numel() < n_min:
        raise ValueError("tensor too small for the packed layout")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """One shell discretization with its tables, factors and workspaces on one GPU."""

    def __init__(self, L, M, m0, N, Ek, Ra, Pr=1.0, dt=200.0, radius_ratio=0.35, device=0, nvec_max=16,
                 refine_fp64=-1, refine_mixed=-1, nr_phys=0, ntheta=0, nphi=0, mixed_solve=0, coriolis=0,
                 graph_capture=0):
        lib = load_library()
        p = _Params(L, M, m0, N, radius_ratio, Ek, Ra, Pr, dt, nr_phys, ntheta, nphi, device, nvec_max,
                    refine_fp64, refine_mixed, mixed_solve, coriolis, int(graph_capture))
        h = ctypes.c_void_p()
        _check(lib.sc_plan_create(ctypes.byref(h), ctypes.byref(p)))
        self._h = h
        lay = _Layout()
        _check(lib.sc_layout(h, ctypes.byref(lay)))
        self.layout = {f: getattr(lay, f) for f, _ in _Layout._fields_}
        self.n_real = lay.n_real

    def close(self):
        if getattr(self, "_h", None):
            _lib.sc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, Ra, Ek, dt):
        _check(_lib.sc_set_params(self._h, Ra, Ek, dt))

    def factor(self, stream=None):
        _check(_lib.sc_factor(self._h, _stream(stream)))

    def step(self, x, C, out, stream=None):
        _check(_lib.sc_step(self._h, _ptr(x, self.n_real), C, _ptr(out, self.n_real), _stream(stream)))
        return out

    def newton_residual(self, x, C, out, stream=None, norm=True):
        rn = ctypes.c_double(0.0)
        _check(_lib.sc_newton_residual(self._h, _ptr(x, self.n_real), C, _ptr(out, self.n_real),
                                       ctypes.byref(rn) if norm else None, _stream(stream)))
        return rn.value if norm else None

    def newton_residual_noalloc(self, x, C, out, rnorm, stream=None):
        """out = B_C(x) - x and rnorm[0] = ||out|| on the device, with no allocation and no
        synchronization (sc_newton_residual_noalloc); rnorm: a float64 CUDA tensor."""
        _check(_lib.sc_newton_residual_noalloc(self._h, _ptr(x, self.n_real), C, _ptr(out, self.n_real),
                                               _ptr(rnorm, 1), _stream(stream)))
        return out

    def tail_ratios(self, x, stream=None):
        """(Chebyshev, spherical-harmonic) tail ratios of a state (sc_tail_ratios)."""
        rc, rl = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(_lib.sc_tail_ratios(self._h, _ptr(x, self.n_real), ctypes.byref(rc), ctypes.byref(rl), _stream(stream)))
        return rc.value, rl.value

    def set_base(self, x, C=0.0, J=-1, stream=None):
        _check(_lib.sc_set_base(self._h, _ptr(x, self.n_real), C, int(J), _stream(stream)))

    def jvp(self, v, out, prec=SC_MIXED, stream=None):
        """v, out: [nvec, n_real] (or [n_real]) float64 CUDA tensors of the same shape."""
        if v.dim() not in (1, 2) or v.shape[-1] != self.n_real:
            raise ValueError("v must be [n_real] or [nvec, n_real]")
        if tuple(out.shape) != tuple(v.shape):
            raise ValueError("out must have the shape of v")
        nvec = 1 if v.dim() == 1 else v.shape[0]
        ld = self.n_real if v.dim() == 1 else v.stride(0)
        ldy = self.n_real if out.dim() == 1 else out.stride(0)
        _check(_lib.sc_jvp(self._h, nvec, _ptr(v, self.n_real * nvec), ld, _ptr(out, self.n_real * nvec), ldy,
                           int(prec), _stream(stream)))
        return out

    def profile(self, enable=True):
        _check(_lib.sc_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total ms, launches)} recorded since the last read; synchronizes."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        _check(_lib.sc_profile_read(self._h, ms, cnt, n))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    def autotune(self, nvec=1, reps=5, stream=None):
        """Times the kernel candidates of the transforms and keeps the fastest (sc_autotune);
        returns the choices and best times."""
        r = _TuneReport()
        _check(_lib.sc_autotune(self._h, int(nvec), int(reps), ctypes.byref(r), _stream(stream)))
        return {"ring_fp32": r.ring_fp32, "ring_fp64": r.ring_fp64, "anal_folded": r.anal_folded,
                "candidates": r.ncand, "ms_fp32": r.ms_fp32, "ms_fp64": r.ms_fp64,
                "linear_mode": bool(r.linear_mode)}

    def set_kernels(self, ring_fp32, ring_fp64, anal_folded):
        """Sets the kernel choices by hand (sc_set_kernels): ring -1 - v register kernel of shape v
        (FP32: 32, 24, 16 rings per workgroup; FP64: 16, 8), k >= 0 LDS kernel with 2^k rings;
        anal_folded 1 or 0."""
        _check(_lib.sc_set_kernels(self._h, int(ring_fp32), int(ring_fp64), int(anal_folded)))

    def kernels(self):
        """The kernel choices in effect (sc_get_kernels)."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.sc_get_kernels(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"ring_fp32": a.value, "ring_fp64": b.value, "anal_folded": c.value}

    def newton(self, x, C=0.0, J=-1, tol=1e-10, gmres_tol=1e-10, restart=40, max_newton=20, max_matvec=400,
               prec=SC_FP64, forcing=None, stream=None):
        """Newton-GMRES in place on x (device); returns (C, report dict)."""
        o = _NewtonOpts(tol, gmres_tol, restart, max_newton, max_matvec, int(prec), int(J),
                        None if forcing is None else _ptr(forcing, self.n_real).value)
        rep = _NewtonReport()
        c = ctypes.c_double(C)
        _check(_lib.sc_newton(self._h, _ptr(x, self.n_real), ctypes.byref(c), ctypes.byref(o), ctypes.byref(rep),
                              _stream(stream)))
        return c.value, _report_dict(rep)


def _report_dict(rep):
    k = rep.newton_steps
    return {"newton_steps": k, "matvecs": rep.matvecs, "converged": bool(rep.converged),
            "rnorm": [rep.rnorm[i] for i in range(k + 1)], "step_matvecs": [rep.step_matvecs[i] for i in range(k)]}


class Batch:
    """A ragged batch of plans whose Jacobian actions run on concurrent stream branches.

    The batch keeps references to its plans; destroy it (close()) before them."""

    def __init__(self, plans):
        lib = load_library()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.sc_batch_create(ctypes.byref(h), arr, len(self.plans)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.sc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def jvp(self, vs, ys, prec=SC_MIXED, stream=None):
        """vs[i], ys[i]: [nvec_i, n_real_i] float64 CUDA tensors of plan i (or None for nvec_i = 0)."""
        n = len(self.plans)
        nv = (ctypes.c_int * n)()
        pv = (ctypes.c_void_p * n)()
        py = (ctypes.c_void_p * n)()
        for i, (p, v, y) in enumerate(zip(self.plans, vs, ys)):
            if v is None:
                nv[i], pv[i], py[i] = 0, None, None
                continue
            k = 1 if v.dim() == 1 else v.shape[0]
            if v.dim() not in (1, 2) or v.shape[-1] != p.n_real:
                raise ValueError("vectors of plan %d must be [n_real] or [nvec, n_real]" % i)
            if y.shape != v.shape:
                raise ValueError("output shape differs from input shape")
            nv[i] = k
            pv[i] = _ptr(v, p.n_real * k).value
            py[i] = _ptr(y, p.n_real * k).value
        _check(_lib.sc_batch_jvp(self._h, nv, pv, py, int(prec), _stream(stream)))
        return ys

    def newton(self, xs, Cs, Js, tol=1e-10, gmres_tol=1e-10, restart=40, max_newton=20, max_matvec=400,
               prec=SC_FP64, forcings=None, stream=None):
        """Newton-GMRES on every plan at once (sc_batch_newton), in place on xs[i] (device);
        returns [(C_i, report dict_i)]."""
        n = len(self.plans)
        px = (ctypes.c_void_p * n)()
        cs = (ctypes.c_double * n)(*[float(c) for c in Cs])
        opts = (_NewtonOpts * n)()
        reps = (_NewtonReport * n)()
        for i, (p, x) in enumerate(zip(self.plans, xs)):
            px[i] = _ptr(x, p.n_real).value
            f = None if forcings is None or forcings[i] is None else _ptr(forcings[i], p.n_real).value
            opts[i] = _NewtonOpts(tol, gmres_tol, restart, max_newton, max_matvec, int(prec), int(Js[i]), f)
        _check(_lib.sc_batch_newton(self._h, px, cs, opts, reps, _stream(stream)))
        return [(cs[i], _report_dict(reps[i])) for i in range(n)]


def _point_dict(pt):
    return {f: getattr(pt, f) for f, _ in _ContPoint._fields_}


def interpolate(src, x, dst, y, stream=None):
    """y (layout of plan dst) = x (layout of plan src) carried to the new grid (sc_interpolate)."""
    _check(_lib.sc_interpolate(src._h, _ptr(x, src.n_real), dst._h, _ptr(y, dst.n_real), _stream(stream)))
    return y


class Continuation:
    """A continuation session (sc_cont_*): Ra (param=SC_CONT_RA) or log10 Ek (SC_CONT_EK) along a
    branch of rotating waves from a converged point of `plan`.  The session may replace the plan
    by finer ones (refinement); state() returns a copy of the newest state."""

    def __init__(self, plan, x0, C0, J, param=SC_CONT_RA, n_opt=4, gamma=50.0, ra_coef=6.5, refine_tol=0.0,
                 refine_growth=1.2, max_retries=3, tol=1e-10, gmres_tol=1e-10, restart=40, max_newton=10,
                 max_matvec=400, prec=SC_FP64, stream=None):
        lib = load_library()
        self.plan = plan
        o = _ContOpts(int(param), int(n_opt), float(gamma), float(ra_coef), float(refine_tol), float(refine_growth),
                      int(max_retries), _NewtonOpts(tol, gmres_tol, restart, max_newton, max_matvec, int(prec),
                                                    int(J), None))
        first = _ContPoint()
        h = ctypes.c_void_p()
        _check(lib.sc_cont_create(ctypes.byref(h), plan._h, _ptr(x0, plan.n_real), float(C0), ctypes.byref(o),
                                  ctypes.byref(first), _stream(stream)))
        self._h = h
        self.first = _point_dict(first)

    def step(self, dp_first=0.0, stream=None):
        pt = _ContPoint()
        _check(_lib.sc_cont_step(self._h, float(dp_first), ctypes.byref(pt), _stream(stream)))
        return _point_dict(pt)

    def layout(self):
        lay = _Layout()
        _check(_lib.sc_cont_layout(self._h, ctypes.byref(lay)))
        return {f: getattr(lay, f) for f, _ in _Layout._fields_}

    def state(self, stream=None):
        """(x, C): a new float64 CUDA tensor with the newest state, and its drift speed."""
        import torch
        n = self.layout()["n_real"]
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        c = ctypes.c_double(0.0)
        _check(_lib.sc_cont_state(self._h, _ptr(x, n), n, ctypes.byref(c), _stream(stream)))
        return x, c.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.sc_cont_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
