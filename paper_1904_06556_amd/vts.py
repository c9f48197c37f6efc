"""Python binding of libvts (include/vts.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory
(tensors are passed by data pointer) and the stream.  Importing this module
loads the in-tree libvts.so and raises if it is missing -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvts.so")

VTS_OK, VTS_EINVAL, VTS_ENOMEM, VTS_EDEVICE, VTS_ESTATE, VTS_ENOTCONV, \
    VTS_ENONDESCENT, VTS_ENONSPD = range(8)
STATUS_NAMES = {0: "VTS_OK", 1: "VTS_EINVAL", 2: "VTS_ENOMEM", 3: "VTS_EDEVICE",
                4: "VTS_ESTATE", 5: "VTS_ENOTCONV", 6: "VTS_ENONDESCENT", 7: "VTS_ENONSPD"}
VTS_FP64, VTS_MIXED = 0, 1
# checkpoint header (vts_get_state): magic, layout version, n_dof, m
STATE_MAGIC, STATE_VERSION, STATE_HEAD = 5657683.0, 2.0, 4

PROF = dict(gs_fine=1, apply_K=2, apply_S=3)
VEC = dict(u=0, rho=1, energy=2, rhs=3, dy=4, g1=5, dnu_lo=6, dnu_hi=7, rho1=8, w=9)


class VtsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem_t(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("levels", C.c_int32),
                ("E", C.c_double), ("nu", C.c_double), ("h", C.c_double),
                ("fixed_host", C.POINTER(C.c_uint8)), ("f_host", C.POINTER(C.c_double)),
                ("V", C.c_double),
                ("rho_lo_host", C.POINTER(C.c_double)), ("rho_hi_host", C.POINTER(C.c_double)),
                ("rho_lo_s", C.c_double), ("rho_hi_s", C.c_double),
                ("precision", C.c_int32), ("nload", C.c_int32)]


class Options_t(C.Structure):
    _fields_ = [("beta", C.c_double), ("gamma", C.c_double), ("p_min", C.c_double),
                ("q_min", C.c_double),
                ("eps_pbm", C.c_double), ("eps_nwt0", C.c_double), ("eps_nwt_min", C.c_double),
                ("eps_nwt_final", C.c_double), ("eps_stat", C.c_double),
                ("accept_stall", C.c_double), ("eps_mr0", C.c_double),
                ("eps_mr_min", C.c_double), ("armijo_c1", C.c_double),
                ("armijo_min", C.c_double), ("max_outer", C.c_int32),
                ("max_newton", C.c_int32), ("max_minres", C.c_int32),
                ("final_res4", C.c_int32), ("p_min_relative", C.c_int32),
                ("stall_steps", C.c_int32), ("use_graphs", C.c_int32),
                ("kkt_tol", C.c_double), ("eps_state", C.c_double), ("log_path", C.c_char_p)]


class LinStats_t(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual", C.c_double)]


class NewtonStats_t(C.Structure):
    _fields_ = [("res_pbm", C.c_double), ("res4", C.c_double), ("kappa", C.c_double),
                ("slope", C.c_double), ("eps_mr", C.c_double), ("minres_its", C.c_int32)]


class PbmStats_t(C.Structure):
    _fields_ = [("gap", C.c_double), ("dual", C.c_double), ("ratio", C.c_double),
                ("stat", C.c_double), ("eps_nwt", C.c_double), ("sum_rho", C.c_double),
                ("newton_its", C.c_int32), ("minres_its", C.c_int32), ("converged", C.c_int32)]


class Result_t(C.Structure):
    _fields_ = [("compliance", C.c_double), ("alpha", C.c_double), ("sum_rho", C.c_double),
                ("res_pbm", C.c_double), ("outer", C.c_int32), ("newton", C.c_int32),
                ("minres", C.c_int32), ("status", C.c_int32),
                ("kkt", C.c_double), ("r_eq", C.c_double), ("r_vol", C.c_double),
                ("r_box", C.c_double), ("r_stat", C.c_double)]


class DocStats_t(C.Structure):
    _fields_ = [("change", C.c_double), ("alpha", C.c_double), ("compliance", C.c_double),
                ("volume", C.c_double), ("bisection_steps", C.c_int32),
                ("minres_its", C.c_int32), ("converged", C.c_int32), ("iterations", C.c_int32)]


class IpOptions_t(C.Structure):
    _fields_ = [("eps_ip", C.c_double), ("sigma_r", C.c_double), ("sigma_s", C.c_double),
                ("r0", C.c_double), ("s0", C.c_double), ("step_frac", C.c_double),
                ("eps_mr0", C.c_double), ("eps_mr_min", C.c_double),
                ("max_iter", C.c_int32), ("max_minres", C.c_int32)]


class IpStats_t(C.Structure):
    _fields_ = [("gap_ratio", C.c_double), ("res_ip", C.c_double), ("compliance", C.c_double),
                ("alpha", C.c_double), ("r", C.c_double), ("s", C.c_double),
                ("kappa_u", C.c_double), ("kappa_nu_lo", C.c_double),
                ("kappa_nu_hi", C.c_double), ("eps_mr", C.c_double),
                ("minres_its", C.c_int32), ("converged", C.c_int32), ("iterations", C.c_int32)]


class RequestInfo_t(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("outer", C.c_int32),
                ("newton", C.c_int32), ("minres", C.c_int32), ("compliance", C.c_double),
                ("alpha", C.c_double), ("sum_rho", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint", C.c_size_t),
                ("n_dof", C.c_int64), ("m", C.c_int64)]


def _struct_dict(s):
    return {k: getattr(s, k) for k, _ in s._fields_}


# the exported entry points and their C signatures
_P, _D = C.c_void_p, C.POINTER(C.c_double)
SIGNATURES = {
    "vts_default_options": (None, [C.POINTER(Options_t)]),
    "vts_create": (C.c_int, [C.POINTER(Problem_t), C.POINTER(Options_t), _P, C.POINTER(_P)]),
    "vts_destroy": (None, [_P]),
    "vts_reset": (C.c_int, [_P]),
    "vts_footprint_bytes": (C.c_size_t, [C.POINTER(Problem_t), C.POINTER(Options_t)]),
    "vts_allocated_bytes": (C.c_size_t, [_P]),
    "vts_sizes": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "vts_set_rho": (C.c_int, [_P, _P]),
    "vts_apply_K": (C.c_int, [_P, _P, _P]),
    "vts_apply_K_f32": (C.c_int, [_P, _P, _P]),
    "vts_apply_K_rho": (C.c_int, [_P, _P, _P, _P]),
    "vts_apply_S_noalloc": (C.c_int, [_P, _P, _P]),
    "vts_apply_K_rho_f32": (C.c_int, [_P, _P, _P, _P]),
    "vts_element_energy": (C.c_int, [_P, _P, _P]),
    "vts_newton_setup": (C.c_int, [_P]),
    "vts_apply_S": (C.c_int, [_P, _P, _P]),
    "vts_precondition": (C.c_int, [_P, _P, _P]),
    "vts_solve_newton": (C.c_int, [_P, C.c_double, C.POINTER(LinStats_t)]),
    "vts_newton_step": (C.c_int, [_P, C.POINTER(NewtonStats_t)]),
    "vts_newton": (C.c_int, [_P, C.c_double, C.c_int32, C.POINTER(NewtonStats_t)]),
    "vts_pbm_iterate": (C.c_int, [_P, C.POINTER(PbmStats_t)]),
    "vts_pbm_solve": (C.c_int, [_P, C.POINTER(Result_t)]),
    "vts_get_vector": (C.c_int, [_P, C.c_int32, _P]),
    "vts_get_state": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    "vts_set_state": (C.c_int, [_P, _P, C.c_size_t]),
    "vts_profile_start": (C.c_int, [_P, C.c_int32]),
    "vts_profile_stop": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    "vts_last_error": (C.c_char_p, [_P]),
    "vts_group_step": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(PbmStats_t)]),
    "vts_doc_step": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double,
                               C.POINTER(DocStats_t)]),
    "vts_doc_solve": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_int32,
                                C.POINTER(DocStats_t)]),
    "vts_ip_default_options": (None, [C.POINTER(IpOptions_t)]),
    "vts_ip_init": (C.c_int, [_P, C.POINTER(IpOptions_t)]),
    "vts_ip_step": (C.c_int, [_P, C.POINTER(IpStats_t)]),
    "vts_ip_solve": (C.c_int, [_P, C.POINTER(IpOptions_t), C.POINTER(IpStats_t)]),
    "vts_server_create": (C.c_int, [C.c_int32, C.c_size_t, C.POINTER(_P)]),
    "vts_server_submit": (C.c_int, [_P, C.POINTER(Problem_t), C.POINTER(Options_t),
                                    C.POINTER(C.c_int64)]),
    "vts_server_poll": (C.c_int32, [_P, C.POINTER(RequestInfo_t), C.c_int32, C.c_double]),
    "vts_server_fetch": (C.c_int, [_P, C.c_int64, _P, _P]),
    "vts_server_clock": (C.c_double, [_P]),
    "vts_server_batching": (C.c_int, [_P, C.c_int32]),
    "vts_server_group_stats": (None, [_P, C.POINTER(C.c_int64)]),
    "vts_server_counts": (None, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "vts_server_destroy": (None, [_P]),
}

_lib = None


def lib():
    """The loaded libvts (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1904_06556_amd.build.build()")
        # torch provides the device memory and streams the library works on:
        # load it first, so that libvts runs on the HIP runtime torch's
        # tensors and streams belong to
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_options(**overrides) -> Options_t:
    o = Options_t()
    lib().vts_default_options(C.byref(o))
    names = {f[0] for f in Options_t._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise KeyError(f"vts_options has no field {k!r}")
        if k == "log_path" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def _ptr(t, dtype, n):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"expected a contiguous {dtype} tensor with >= {n} elements")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return C.c_void_p(None)        # host-side validation still runs
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _problem_struct(nx, ny, nz, levels, fixed, f, V, rho_lo, rho_hi, E, nu, h, precision,
                    nload=1):
    """vts_problem over host arrays; returns it with the arrays it points to
    (f: nload load cases of n_dof entries each, one after another)."""
    fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.size != max(int(nload), 1) * fixed.size:
        raise ValueError("f must hold nload x n_dof entries")
    pr = Problem_t()
    pr.nx, pr.ny, pr.nz, pr.levels = nx, ny, nz, levels
    pr.E, pr.nu, pr.h, pr.V = E, nu, h, V
    pr.fixed_host = fixed.ctypes.data_as(C.POINTER(C.c_uint8))
    pr.f_host = f.ctypes.data_as(C.POINTER(C.c_double))
    keep = [fixed, f]
    if np.ndim(rho_lo):
        lo = np.ascontiguousarray(rho_lo, dtype=np.float64)
        pr.rho_lo_host = lo.ctypes.data_as(_D)
        keep.append(lo)
    else:
        pr.rho_lo_s = float(rho_lo)
    if np.ndim(rho_hi):
        hi = np.ascontiguousarray(rho_hi, dtype=np.float64)
        pr.rho_hi_host = hi.ctypes.data_as(_D)
        keep.append(hi)
    else:
        pr.rho_hi_s = float(rho_hi)
    pr.precision = precision
    pr.nload = nload
    return pr, keep


class Context:
    """One problem's device state (vts_ctx)."""

    def __init__(self, nx, ny, nz, levels, fixed, f, V, rho_lo=1e-3, rho_hi=1.0, E=1.0,
                 nu=0.3, h=1.0, precision=VTS_FP64, options: Optional[Options_t] = None,
                 stream=None, nload=1):
        L = lib()
        pr, self._keep = _problem_struct(nx, ny, nz, levels, fixed, f, V, rho_lo, rho_hi, E, nu,
                                         h, precision, nload)
        self._pr = pr
        self._opt = options if options is not None else default_options()
        self.stream = stream
        h_ = C.c_void_p()
        st = L.vts_create(C.byref(pr), C.byref(self._opt), _stream(stream), C.byref(h_))
        if st != VTS_OK:
            raise VtsError(st, L.vts_last_error(None).decode())
        self.h = h_
        nd, m, nf, lv = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        L.vts_sizes(self.h, C.byref(nd), C.byref(m), C.byref(nf), C.byref(lv))
        self.n_dof, self.m, self.n_free, self.levels = nd.value, m.value, nf.value, lv.value
        # load cases: displacement-sized vectors hold nload n_dof entries
        self.nload = max(int(nload), 1)
        self.n_vec = self.nload * self.n_dof

    @classmethod
    def from_problem(cls, pr, precision=None, options=None, stream=None):
        """A problem with load cases (extra["load_cases"], k x n_dof) gives a
        context with nload = k; otherwise its load f."""
        cases = pr.extra.get("load_cases")
        if precision is None:
            precision = VTS_MIXED if pr.extra.get("precision") == "mixed" else VTS_FP64
        if cases is not None and len(cases) > 1:
            f = np.ascontiguousarray(np.asarray(cases, dtype=np.float64).ravel())
            return cls(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, f, pr.V, pr.rho_lo, pr.rho_hi,
                       pr.E, pr.nu, pr.h, precision, options, stream, nload=len(cases))
        return cls(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, pr.f, pr.V, pr.rho_lo, pr.rho_hi,
                   pr.E, pr.nu, pr.h, precision, options, stream)

    @staticmethod
    def footprint_bytes(nx, ny, nz, levels, precision=VTS_FP64) -> int:
        pr = Problem_t()
        pr.nx, pr.ny, pr.nz, pr.levels = nx, ny, nz, levels
        pr.E, pr.nu, pr.h = 1.0, 0.3, 1.0
        dummy_u8 = (C.c_uint8 * 1)()
        dummy_d = (C.c_double * 1)()
        pr.fixed_host = C.cast(dummy_u8, C.POINTER(C.c_uint8))
        pr.f_host = C.cast(dummy_d, _D)
        pr.precision = precision
        return int(lib().vts_footprint_bytes(C.byref(pr), None))

    def allocated_bytes(self) -> int:
        return int(lib().vts_allocated_bytes(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().vts_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != VTS_OK:
            raise VtsError(st, lib().vts_last_error(self.h).decode())

    def reset(self):
        self._check(lib().vts_reset(self.h))

    # --- operators -------------------------------------------------------
    def set_rho(self, rho):
        import torch
        self._check(lib().vts_set_rho(self.h, _ptr(rho, torch.float64, self.m)))

    def apply_K(self, x, y):
        import torch
        self._check(lib().vts_apply_K(self.h, _ptr(x, torch.float64, self.n_vec),
                                      _ptr(y, torch.float64, self.n_vec)))

    def apply_K_f32(self, x, y):
        import torch
        self._check(lib().vts_apply_K_f32(self.h, _ptr(x, torch.float32, self.n_dof),
                                          _ptr(y, torch.float32, self.n_dof)))

    def apply_K_rho(self, rho, x, y):
        import torch
        self._check(lib().vts_apply_K_rho(self.h, _ptr(rho, torch.float64, self.m),
                                          _ptr(x, torch.float64, self.n_vec),
                                          _ptr(y, torch.float64, self.n_vec)))

    def apply_K_rho_f32(self, rho, x, y):
        import torch
        self._check(lib().vts_apply_K_rho_f32(self.h, _ptr(rho, torch.float32, self.m),
                                              _ptr(x, torch.float32, self.n_dof),
                                              _ptr(y, torch.float32, self.n_dof)))

    def element_energy(self, u, e):
        import torch
        self._check(lib().vts_element_energy(self.h, _ptr(u, torch.float64, self.n_vec),
                                             _ptr(e, torch.float64, self.m)))

    def newton_setup(self):
        self._check(lib().vts_newton_setup(self.h))

    def apply_S(self, x, y):
        import torch
        self._check(lib().vts_apply_S(self.h, _ptr(x, torch.float64, self.n_vec + 1),
                                      _ptr(y, torch.float64, self.n_vec + 1)))

    def apply_S_noalloc(self, x, y):
        import torch
        self._check(lib().vts_apply_S_noalloc(self.h, _ptr(x, torch.float64, self.n_dof + 1),
                                              _ptr(y, torch.float64, self.n_dof + 1)))

    def precondition(self, r, z):
        import torch
        self._check(lib().vts_precondition(self.h, _ptr(r, torch.float64, self.n_vec + 1),
                                           _ptr(z, torch.float64, self.n_vec + 1)))

    # --- solvers ---------------------------------------------------------
    def solve_newton(self, eps_mr):
        s = LinStats_t()
        self._check(lib().vts_solve_newton(self.h, eps_mr, C.byref(s)))
        return _struct_dict(s)

    def newton_step(self):
        s = NewtonStats_t()
        self._check(lib().vts_newton_step(self.h, C.byref(s)))
        return _struct_dict(s)

    def newton(self, eps_nwt, final=False):
        s = NewtonStats_t()
        self._check(lib().vts_newton(self.h, eps_nwt, int(final), C.byref(s)))
        return _struct_dict(s)

    def pbm_iterate(self):
        s = PbmStats_t()
        self._check(lib().vts_pbm_iterate(self.h, C.byref(s)))
        return _struct_dict(s)

    def pbm_solve(self, check=True):
        r = Result_t()
        st = lib().vts_pbm_solve(self.h, C.byref(r))
        if check:
            self._check(st)
        return _struct_dict(r)

    # --- damped optimality criteria (Algorithm 4) -------------------------
    def doc_step(self, q=0.5, tau=1e-4, eps_doc=-1.0, eps_mr=1e-6):
        s = DocStats_t()
        self._check(lib().vts_doc_step(self.h, q, tau, eps_doc, eps_mr, C.byref(s)))
        return _struct_dict(s)

    def doc_solve(self, q=0.5, eps_doc=1e-3, eps_mr=1e-6, max_iter=1000, check=True):
        s = DocStats_t()
        st = lib().vts_doc_solve(self.h, q, eps_doc, eps_mr, max_iter, C.byref(s))
        if check:
            self._check(st)
        return dict(_struct_dict(s), status=st)

    # --- primal-dual interior point method (Algorithm 3) -----------------
    @staticmethod
    def ip_options(**kw):
        o = IpOptions_t()
        lib().vts_ip_default_options(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def ip_init(self, **kw):
        self._check(lib().vts_ip_init(self.h, C.byref(self.ip_options(**kw))))

    def ip_step(self, check=True):
        s = IpStats_t()
        st = lib().vts_ip_step(self.h, C.byref(s))
        if check:
            self._check(st)
        return dict(_struct_dict(s), status=st)

    def ip_solve(self, check=True, **kw):
        s = IpStats_t()
        st = lib().vts_ip_solve(self.h, C.byref(self.ip_options(**kw)), C.byref(s))
        if check:
            self._check(st)
        return dict(_struct_dict(s), status=st)

    # --- profiling -------------------------------------------------------
    def profile_start(self, kernel_class):
        k = PROF[kernel_class] if isinstance(kernel_class, str) else kernel_class
        self._check(lib().vts_profile_start(self.h, k))

    def profile_stop(self):
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        self._check(lib().vts_profile_stop(self.h, C.byref(ms), C.byref(n), C.byref(b)))
        return dict(total_ms=ms.value, launches=n.value, bytes=b.value)

    # --- state -----------------------------------------------------------
    def get_vector(self, which, out):
        import torch
        n = {0: self.n_vec, 1: self.m, 2: self.m, 3: self.n_vec + 1, 4: self.n_vec + 1,
             5: self.n_vec, 6: self.m, 7: self.m, 8: self.m, 9: self.m}[VEC.get(which, which)
                                                                      if isinstance(which, str) else which]
        w = VEC[which] if isinstance(which, str) else which
        self._check(lib().vts_get_vector(self.h, w, _ptr(out, torch.float64, n)))

    def vector(self, which):
        import torch
        w = VEC[which] if isinstance(which, str) else which
        n = {0: self.n_vec, 1: self.m, 2: self.m, 3: self.n_vec + 1, 4: self.n_vec + 1,
             5: self.n_vec, 6: self.m, 7: self.m, 8: self.m, 9: self.m}[w]
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        self.get_vector(w, out)
        torch.cuda.synchronize()
        return out

    def get_state(self) -> np.ndarray:
        nb = C.c_size_t(0)
        self._check(lib().vts_get_state(self.h, None, C.byref(nb)))
        buf = np.empty(nb.value // 8, dtype=np.float64)
        self._check(lib().vts_get_state(self.h, buf.ctypes.data_as(C.c_void_p), C.byref(nb)))
        return buf

    def set_state(self, buf: np.ndarray):
        b = np.ascontiguousarray(buf, dtype=np.float64)
        self._check(lib().vts_set_state(self.h, b.ctypes.data_as(C.c_void_p), b.nbytes))

    def state_dict(self):
        """Unpacks get_state() by the layout documented in vts.h."""
        b = self.get_state()
        nd, m = self.n_vec, self.m
        o = STATE_HEAD
        out = {"u": b[o:o + nd], "alpha": b[o + nd]}
        o += nd + 1
        for name in ("nu_lo", "nu_hi", "rho", "mu_lo", "mu_hi", "p", "q_lo", "q_hi"):
            out[name] = b[o:o + m]
            o += m
        out["eps_nwt"], out["eps_mr"] = b[o], b[o + 1]
        out["outer"], out["newton"], out["minres"] = (int(b[o + 2]), int(b[o + 3]),
                                                      int(b[o + 4]))
        return out

    @staticmethod
    def pack_state(d, n_dof, m):
        """Packs a state dict into the checkpoint layout; the counters
        (outer, newton, minres) default to 0.  n_dof is the length of u
        (n_vec, load cases times n_dof, for several load cases)."""
        parts = [[STATE_MAGIC, STATE_VERSION, n_dof, m], np.asarray(d["u"], float), [d["alpha"]]]
        for name in ("nu_lo", "nu_hi", "rho", "mu_lo", "mu_hi", "p", "q_lo", "q_hi"):
            parts.append(np.asarray(d[name], float))
        parts.append([d["eps_nwt"], d["eps_mr"], d.get("outer", 0), d.get("newton", 0),
                      d.get("minres", 0)])
        return np.concatenate(parts)


def group_step(contexts):
    """One outer PBM iteration of each context, overlapping on the device
    (vts_group_step); returns the per-context statistics."""
    k = len(contexts)
    hs = (_P * k)(*[c.h for c in contexts])
    st = (PbmStats_t * k)()
    code = lib().vts_group_step(hs, k, st)
    if code != VTS_OK:
        raise VtsError(code, "vts_group_step")
    return [_struct_dict(st[i]) for i in range(k)]


class Server:
    """Request loop for independent VTS problems (vts_server): a device pool
    of hbm_bytes, `slots` workers with one stream each, admission by
    footprint."""

    def __init__(self, slots: int, hbm_bytes: int, batching: bool = True):
        h_ = C.c_void_p()
        st = lib().vts_server_create(int(slots), int(hbm_bytes), C.byref(h_))
        if st != VTS_OK:
            raise VtsError(st, "vts_server_create")
        self.h = h_
        if not batching:
            st = lib().vts_server_batching(self.h, 0)
            if st != VTS_OK:
                raise VtsError(st, "vts_server_batching")

    def group_stats(self):
        """Counters of the same-shape MINRES group runners (summed)."""
        a = (C.c_int64 * 5)()
        lib().vts_server_group_stats(self.h, a)
        return dict(steps=a[0], solves=a[1], kernel_ops=a[2], launches=a[3], max_batch=a[4],
                    mean_batch=(a[2] / a[3]) if a[3] else None)

    def submit(self, pr, precision=None, options: Optional[Options_t] = None) -> int:
        if precision is None:
            precision = VTS_MIXED if pr.extra.get("precision") == "mixed" else VTS_FP64
        ps, keep = _problem_struct(pr.nx, pr.ny, pr.nz, pr.levels, pr.fixed, pr.f, pr.V,
                                   pr.rho_lo, pr.rho_hi, pr.E, pr.nu, pr.h, precision)
        rid = C.c_int64()
        st = lib().vts_server_submit(self.h, C.byref(ps),
                                     C.byref(options) if options is not None else None,
                                     C.byref(rid))
        del keep                                  # the server copied the arrays
        if st != VTS_OK:
            raise VtsError(st, "vts_server_submit")
        return rid.value

    def poll(self, timeout_s: float = 0.0, max_n: int = 64):
        buf = (RequestInfo_t * max_n)()
        n = lib().vts_server_poll(self.h, buf, max_n, float(timeout_s))
        return [_struct_dict(buf[i]) for i in range(n)]

    def fetch(self, rid: int, m: int, n_dof: int):
        rho = np.empty(m)
        u = np.empty(n_dof)
        st = lib().vts_server_fetch(self.h, int(rid), rho.ctypes.data_as(C.c_void_p),
                                    u.ctypes.data_as(C.c_void_p))
        if st != VTS_OK:
            raise VtsError(st, f"vts_server_fetch({rid})")
        return rho, u

    def clock(self) -> float:
        return float(lib().vts_server_clock(self.h))

    def counts(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        lib().vts_server_counts(self.h, C.byref(a), C.byref(b), C.byref(c))
        return dict(pending=a.value, running=b.value, finished=c.value)

    def close(self):
        if getattr(self, "h", None):
            lib().vts_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
