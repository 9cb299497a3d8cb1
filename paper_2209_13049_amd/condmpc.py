"""ctypes binding of libcondmpc.so (include/condmpc.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
Host arrays are numpy float64; device arrays are torch CUDA (HIP) tensors, which own the
memory, and work is issued on torch's current stream.  If the shared library is missing
every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcondmpc.so")

OK, MAX_ITER, SMALL_STEP = 0, 1, 2
ERR_INVALID, ERR_NONFINITE, ERR_X0_BOUNDS, ERR_CHOLESKY, ERR_HIP, ERR_NOMEM = -1, -2, -3, -4, -5, -6
FP64, FP32_SYRK, BF16_SYRK = 0, 1, 2

# every function declared in include/condmpc.h
EXPORTS = [
    "cmpc_default_options", "cmpc_problem_create", "cmpc_problem_destroy", "cmpc_problem_dims",
    "cmpc_problem_info", "cmpc_set_x0", "cmpc_solve", "cmpc_get_solution", "cmpc_get_iterate", "cmpc_export_dense",
    "cmpc_form_condensed", "cmpc_newton_step", "cmpc_potrf", "cmpc_potrs", "cmpc_last_error",
    "cmpc_status_str",
]

_dp = ctypes.POINTER(ctypes.c_double)


class LQDesc(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nu", ctypes.c_int), ("N", ctypes.c_int),
                ("A", _dp), ("B", _dp), ("Q", _dp), ("R", _dp), ("Qf", _dp),
                ("xl", _dp), ("xu", _dp), ("ul", _dp), ("uu", _dp)]


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_refine", ctypes.c_int),
                ("mu_switch", ctypes.c_double), ("check_every", ctypes.c_int),
                ("profile", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("precision_switch_iter", ctypes.c_int), ("refine_steps", ctypes.c_int),
                ("obj", ctypes.c_double), ("primal_res", ctypes.c_double),
                ("dual_res", ctypes.c_double), ("compl_res", ctypes.c_double),
                ("mu", ctypes.c_double), ("gap", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_syrk", ctypes.c_double),
                ("ms_form", ctypes.c_double), ("ms_potrf", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("mx", ctypes.c_int), ("m", ctypes.c_int),
                ("gamma_nnz", ctypes.c_longlong), ("syrk_flops", ctypes.c_double),
                ("potrf_flops", ctypes.c_double), ("syrk_workgroups", ctypes.c_int),
                ("syrk_partial_slots", ctypes.c_int), ("device_bytes", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2209_13049_amd.build")
    lib = ctypes.CDLL(path)
    vp, ip, i = ctypes.c_void_p, ctypes.c_int, ctypes.c_int
    sig = {
        "cmpc_default_options": (None, [ctypes.POINTER(Options)]),
        "cmpc_problem_create": (i, [ctypes.POINTER(LQDesc), vp, ctypes.POINTER(vp)]),
        "cmpc_problem_destroy": (None, [vp]),
        "cmpc_problem_dims": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]),
        "cmpc_problem_info": (i, [vp, ctypes.POINTER(Info)]),
        "cmpc_set_x0": (i, [vp, vp, i]),
        "cmpc_solve": (i, [vp, ctypes.POINTER(Options), ctypes.POINTER(Result)]),
        "cmpc_get_solution": (i, [vp, vp, vp, i]),
        "cmpc_get_iterate": (i, [vp, vp, vp, vp, vp, i]),
        "cmpc_export_dense": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "cmpc_form_condensed": (i, [vp, vp, vp, i]),
        "cmpc_newton_step": (i, [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp,
                                 vp, vp, vp]),
        "cmpc_potrf": (i, [vp, i, i, vp, ctypes.POINTER(i)]),
        "cmpc_potrs": (i, [vp, i, i, vp, vp]),
        "cmpc_last_error": (ctypes.c_char_p, []),
        "cmpc_status_str": (ctypes.c_char_p, [i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class CmpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"condmpc error {code}: {msg}")
        self.code = code


def _check(rc, allow_positive=False):
    if rc < 0 or (rc > 0 and not allow_positive):
        raise CmpcError(rc, load().cmpc_last_error().decode())
    return rc


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    """Device pointer of a contiguous float64 torch CUDA tensor."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def default_options(**kw) -> Options:
    o = Options()
    load().cmpc_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Problem:
    """A reduced LQ-MPC problem resident on the GPU (wraps cmpc_problem)."""

    def __init__(self, prob, stream=None):
        lib = load()
        self._keep = [_f64(prob.A), _f64(prob.B), _f64(prob.Q), _f64(prob.R), _f64(prob.Qf),
                      _f64(prob.xl), _f64(prob.xu), _f64(prob.ul), _f64(prob.uu)]
        A, B, Q, R, Qf, xl, xu, ul, uu = self._keep
        d = LQDesc(ns=A.shape[0], nu=B.shape[1], N=int(prob.N), A=_ptr(A), B=_ptr(B),
                   Q=_ptr(Q), R=_ptr(R), Qf=_ptr(Qf), xl=_ptr(xl), xu=_ptr(xu), ul=_ptr(ul),
                   uu=_ptr(uu))
        self._h = ctypes.c_void_p()
        st = _stream() if stream is None else ctypes.c_void_p(stream)
        _check(lib.cmpc_problem_create(ctypes.byref(d), st, ctypes.byref(self._h)))
        n, mx, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.cmpc_problem_dims(self._h, ctypes.byref(n), ctypes.byref(mx), ctypes.byref(m)))
        self.n, self.mx, self.m = n.value, mx.value, m.value
        self.ns, self.nu, self.N = A.shape[0], B.shape[1], int(prob.N)

    def info(self) -> dict:
        inf = Info()
        _check(load().cmpc_problem_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def close(self):
        if self._h:
            load().cmpc_problem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_x0(self, x0):
        import torch
        if isinstance(x0, torch.Tensor):
            return _check(load().cmpc_set_x0(self._h, _dev(x0), 1))
        x = _f64(x0)
        return _check(load().cmpc_set_x0(self._h, x.ctypes.data_as(ctypes.c_void_p), 0))

    def solve(self, **opts) -> dict:
        o = default_options(**opts)
        r = Result()
        rc = load().cmpc_solve(self._h, ctypes.byref(o), ctypes.byref(r))
        _check(rc, allow_positive=True)
        return r.as_dict()

    def solve_raw(self, options: Options, result: Result) -> int:
        return load().cmpc_solve(self._h, ctypes.byref(options), ctypes.byref(result))

    def solution(self, with_x=True):
        u = np.empty(self.n)
        x = np.empty(self.mx) if with_x else None
        _check(load().cmpc_get_solution(self._h, u.ctypes.data_as(ctypes.c_void_p),
                                        x.ctypes.data_as(ctypes.c_void_p) if with_x else None, 0))
        return u, x

    def iterate(self):
        v, s, lam, z = (np.empty(self.n), np.empty(self.m), np.empty(self.m), np.empty(self.m))
        vp = ctypes.c_void_p
        _check(load().cmpc_get_iterate(self._h, *(vp(a.ctypes.data) for a in (v, s, lam, z)), 0))
        return v, s, lam, z

    def export_dense(self, gamma=True, x0_data=True):
        H = np.empty((self.n, self.n))
        out = {"H": H}
        vp = ctypes.c_void_p
        args = [vp(H.ctypes.data)]
        if x0_data:
            h, h0, d, c = np.empty(self.n), np.empty(1), np.empty(self.m), np.empty(self.mx)
            out.update(h=h, h0=h0, d=d, c=c)
            args += [vp(a.ctypes.data) for a in (h, h0, d, c)]
        else:
            args += [None, None, None, None]
        if gamma:
            G = np.empty((self.mx, self.n))
            out["Gamma"] = G
            args.append(vp(G.ctypes.data))
        else:
            args.append(None)
        _check(load().cmpc_export_dense(self._h, *args))
        if x0_data:
            out["h0"] = float(out["h0"][0])
        return out

    def form_condensed(self, sigma, K, precision=FP64):
        """K (n x n float64 CUDA tensor) <- lower triangle of H + J' diag(sigma) J."""
        return _check(load().cmpc_form_condensed(self._h, _dev(sigma), _dev(K), precision))

    def newton_step(self, v, s, lam, z, mu, tau):
        import torch
        pv = torch.empty(self.n, dtype=torch.float64, device=v.device)
        ps, plam, pz = (torch.empty(self.m, dtype=torch.float64, device=v.device) for _ in range(3))
        al = np.zeros(2)
        _check(load().cmpc_newton_step(self._h, _dev(v), _dev(s), _dev(lam), _dev(z), float(mu),
                                       float(tau), _dev(pv), _dev(ps), _dev(plam), _dev(pz),
                                       al.ctypes.data_as(ctypes.c_void_p)))
        return dict(pv=pv, ps=ps, plam=plam, pz=pz, alpha=float(al[0]), alpha_z=float(al[1]))


def potrf(K, ld=None):
    """In-place Cholesky of the lower triangle of a float64 CUDA tensor (n x ld)."""
    n = K.shape[0]
    info = ctypes.c_int(0)
    rc = load().cmpc_potrf(_dev(K), n, ld or K.shape[1], _stream(), ctypes.byref(info))
    _check(rc)
    return info.value


def potrs(L, b, ld=None):
    n = L.shape[0]
    return _check(load().cmpc_potrs(_dev(L), n, ld or L.shape[1], _dev(b), _stream()))


def status_str(code: int) -> str:
    return load().cmpc_status_str(code).decode()
