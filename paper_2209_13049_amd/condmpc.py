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
POTRF_NOALLOC_MAX_N = 4096
MLP_BF16, MLP_FP32 = 0, 1

# every function declared in include/condmpc.h
EXPORTS = [
    "cmpc_default_options", "cmpc_problem_create", "cmpc_problem_destroy", "cmpc_problem_dims",
    "cmpc_problem_info", "cmpc_set_x0", "cmpc_solve", "cmpc_solve_warm", "cmpc_get_solution", "cmpc_get_iterate", "cmpc_export_dense",
    "cmpc_form_condensed", "cmpc_newton_step", "cmpc_potrf", "cmpc_potrf_noalloc", "cmpc_potrs", "cmpc_batch_create",
    "cmpc_batch_destroy", "cmpc_batch_size", "cmpc_batch_instance", "cmpc_batch_solve",
    "cmpc_batch_solve_warm", "cmpc_mlp_set_fallback",
    "cmpc_batch_tune", "cmpc_tune_lookup", "cmpc_tune_store", "cmpc_tune_clear", "cmpc_default_train_opts",
    "cmpc_mlp_create", "cmpc_mlp_destroy", "cmpc_mlp_param_count", "cmpc_mlp_get_params",
    "cmpc_mlp_set_params", "cmpc_mlp_gradients", "cmpc_mlp_train", "cmpc_mlp_predict",
    "cmpc_judge", "cmpc_surrogate_solve", "cmpc_last_error", "cmpc_status_str",
]

_dp = ctypes.POINTER(ctypes.c_double)


class LQDesc(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nu", ctypes.c_int), ("N", ctypes.c_int),
                ("A", _dp), ("B", _dp), ("Q", _dp), ("R", _dp), ("Qf", _dp),
                ("xl", _dp), ("xu", _dp), ("ul", _dp), ("uu", _dp),
                ("nc", ctypes.c_int), ("S", _dp), ("E", _dp), ("F", _dp), ("gl", _dp),
                ("gu", _dp), ("w", _dp), ("Kfb", _dp), ("data_on_device", ctypes.c_int)]


LOG_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_refine", ctypes.c_int),
                ("mu_switch", ctypes.c_double), ("check_every", ctypes.c_int),
                ("profile", ctypes.c_int), ("equilibrate", ctypes.c_int),
                ("refine_contract", ctypes.c_double), ("log", LOG_FN),
                ("log_ctx", ctypes.c_void_p), ("warm_mu", ctypes.c_double)]


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


class TuneReport(ctypes.Structure):
    _fields_ = [("quantum", ctypes.c_int), ("persistent", ctypes.c_int),
                ("candidates", ctypes.c_int), ("syrk_us", ctypes.c_double),
                ("default_us", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TrainOpts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("epochs", ctypes.c_int), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("weight_decay", ctypes.c_float)]


class SurrogateReport(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("accepted", ctypes.c_int),
                ("fallback_solved", ctypes.c_int), ("fallback_failed", ctypes.c_int),
                ("max_violation_accepted", ctypes.c_double),
                ("max_gap_accepted", ctypes.c_double), ("ms_infer", ctypes.c_double),
                ("ms_judge", ctypes.c_double), ("ms_fallback", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

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
        "cmpc_solve_warm": (i, [vp, ctypes.POINTER(Options), vp, i, ctypes.POINTER(Result)]),
        "cmpc_get_solution": (i, [vp, vp, vp, i]),
        "cmpc_get_iterate": (i, [vp, vp, vp, vp, vp, i]),
        "cmpc_export_dense": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "cmpc_form_condensed": (i, [vp, vp, vp, i]),
        "cmpc_newton_step": (i, [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp,
                                 vp, vp, vp]),
        "cmpc_potrf": (i, [vp, i, i, vp, ctypes.POINTER(i)]),
        "cmpc_potrf_noalloc": (i, [vp, i, i, vp, ctypes.POINTER(i)]),
        "cmpc_potrs": (i, [vp, i, i, vp, vp]),
        "cmpc_batch_create": (i, [i, ctypes.POINTER(LQDesc), ctypes.POINTER(_dp), vp,
                                  ctypes.POINTER(vp)]),
        "cmpc_batch_destroy": (None, [vp]),
        "cmpc_batch_size": (i, [vp]),
        "cmpc_batch_instance": (vp, [vp, i]),
        "cmpc_batch_solve": (i, [vp, ctypes.POINTER(Options), ctypes.POINTER(Result)]),
        "cmpc_batch_solve_warm": (i, [vp, ctypes.POINTER(Options), ctypes.POINTER(vp), i,
                                      ctypes.POINTER(Result)]),
        "cmpc_mlp_set_fallback": (i, [vp, vp, i]),
        "cmpc_batch_tune": (i, [vp, i, ctypes.POINTER(TuneReport)]),
        "cmpc_tune_lookup": (i, [i, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "cmpc_tune_store": (i, [i, i, i, i, i]),
        "cmpc_tune_clear": (None, []),
        "cmpc_default_train_opts": (None, [ctypes.POINTER(TrainOpts)]),
        "cmpc_mlp_create": (i, [vp, i, i, i, vp, ctypes.POINTER(vp)]),
        "cmpc_mlp_destroy": (None, [vp]),
        "cmpc_mlp_param_count": (ctypes.c_longlong, [vp]),
        "cmpc_mlp_get_params": (i, [vp, vp]),
        "cmpc_mlp_set_params": (i, [vp, vp]),
        "cmpc_mlp_gradients": (i, [vp, vp, vp, i, vp, vp, vp]),
        "cmpc_mlp_train": (i, [vp, vp, vp, i, ctypes.POINTER(TrainOpts), vp, vp]),
        "cmpc_mlp_predict": (i, [vp, vp, i, vp]),
        "cmpc_judge": (i, [vp, vp, vp, i, vp, vp, vp, vp]),
        "cmpc_surrogate_solve": (i, [vp, vp, i, vp, vp, ctypes.POINTER(SurrogateReport)]),
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


def _desc(prob):
    """LQDesc of an LQProblem and the host arrays it points into (keep them alive)."""
    keep = [_f64(prob.A), _f64(prob.B), _f64(prob.Q), _f64(prob.R), _f64(prob.Qf),
            _f64(prob.xl), _f64(prob.xu), _f64(prob.ul), _f64(prob.uu)]
    A, B, Q, R, Qf, xl, xu, ul, uu = keep
    d = LQDesc(ns=A.shape[0], nu=B.shape[1], N=int(prob.N), A=_ptr(A), B=_ptr(B), Q=_ptr(Q),
               R=_ptr(R), Qf=_ptr(Qf), xl=_ptr(xl), xu=_ptr(xu), ul=_ptr(ul), uu=_ptr(uu))
    for name in ("S", "E", "F", "gl", "gu", "w", "Kfb"):
        a = getattr(prob, name, None)
        if a is not None:
            a = _f64(a)
            keep.append(a)
            setattr(d, name, _ptr(a))
    if getattr(prob, "E", None) is not None:
        d.nc = int(np.shape(prob.E)[0])
    return d, keep


def _desc_device(prob):
    """The same descriptor with every array in device memory (data_on_device = 1)."""
    import torch
    d, keep = _desc(prob)
    dev = []
    for name, _ in LQDesc._fields_:
        ptr = getattr(d, name)
        if isinstance(ptr, _dp) and ptr:
            a = next(k for k in keep if k.ctypes.data == ctypes.cast(ptr, ctypes.c_void_p).value)
            t = torch.from_numpy(a).to("cuda")
            dev.append(t)
            setattr(d, name, ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp))
    d.data_on_device = 1
    return d, keep + dev


class Problem:
    """A reduced LQ-MPC problem resident on the GPU (wraps cmpc_problem).  device_data: hand
    the library device copies of the data (data_on_device = 1)."""

    def __init__(self, prob, stream=None, _handle=None, device_data=False):
        lib = load()
        self._borrowed = _handle is not None
        if _handle is None:
            d, self._keep = _desc_device(prob) if device_data else _desc(prob)
            self._h = ctypes.c_void_p()
            st = _stream() if stream is None else ctypes.c_void_p(stream)
            _check(lib.cmpc_problem_create(ctypes.byref(d), st, ctypes.byref(self._h)))
        else:
            self._h = ctypes.c_void_p(_handle)
        n, mx, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.cmpc_problem_dims(self._h, ctypes.byref(n), ctypes.byref(mx), ctypes.byref(m)))
        self.n, self.mx, self.m = n.value, mx.value, m.value
        self.ns, self.nu, self.N = int(np.shape(prob.A)[0]), int(np.shape(prob.B)[1]), int(prob.N)

    def info(self) -> dict:
        inf = Info()
        _check(load().cmpc_problem_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def close(self):
        if self._h and not self._borrowed:
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

    def solve(self, log=None, **opts) -> dict:
        """Algorithm 1 from the start point; log: callable receiving one line (str) per
        iteration and one at the end."""
        o = default_options(**opts)
        if log is not None:
            fn = LOG_FN(lambda line, ctx: log(line.decode()))
            o.log = fn                      # referenced by `fn` for the duration of the call
        r = Result()
        rc = load().cmpc_solve(self._h, ctypes.byref(o), ctypes.byref(r))
        _check(rc, allow_positive=True)
        return r.as_dict()

    def solve_raw(self, options: Options, result: Result) -> int:
        return load().cmpc_solve(self._h, ctypes.byref(options), ctypes.byref(result))

    def solve_warm(self, v0=None, **opts) -> dict:
        """cmpc_solve_warm: Algorithm 1 from the controls v0 (numpy array or float64 CUDA
        tensor), or with v0 None from the last solution shifted one stage (receding horizon)."""
        import torch
        o = default_options(**opts)
        r = Result()
        if v0 is None:
            rc = load().cmpc_solve_warm(self._h, ctypes.byref(o), None, 0, ctypes.byref(r))
        elif isinstance(v0, torch.Tensor):
            rc = load().cmpc_solve_warm(self._h, ctypes.byref(o), _dev(v0), 1, ctypes.byref(r))
        else:
            v = _f64(v0)
            rc = load().cmpc_solve_warm(self._h, ctypes.byref(o), v.ctypes.data_as(ctypes.c_void_p),
                                        0, ctypes.byref(r))
        _check(rc, allow_positive=True)
        return r.as_dict()

    def solution(self, with_x=True):
        """(u, x): the inputs u_t = K x_t + v_t (= v without a feedback) and the states
        x_1..x_N (ns N, the problem's own states)."""
        u = np.empty(self.n)
        x = np.empty(self.ns * self.N) if with_x else None
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


class Batch:
    """Independent problems of uneven size solved together (wraps cmpc_batch).

    probs: LQProblems; their x0 is set at creation unless with_x0 is False.  Instance i is
    available as batch[i], a Problem sharing the batch's device memory (valid until close).
    """

    def __init__(self, probs, with_x0=True, stream=None):
        lib = load()
        probs = list(probs)
        self.count = len(probs)
        descs = (LQDesc * self.count)()
        self._keep = []
        x0p = (_dp * self.count)()
        for i, pr in enumerate(probs):
            d, keep = _desc(pr)
            descs[i] = d
            self._keep.append(keep)
            if with_x0 and pr.x0 is not None:
                x0 = _f64(pr.x0)
                self._keep.append(x0)
                x0p[i] = _ptr(x0)
        self._h = ctypes.c_void_p()
        st = _stream() if stream is None else ctypes.c_void_p(stream)
        _check(lib.cmpc_batch_create(self.count, descs, x0p, st, ctypes.byref(self._h)))
        self.instances = []
        for i, pr in enumerate(probs):
            h = lib.cmpc_batch_instance(self._h, i)
            if not h:
                raise CmpcError(ERR_INVALID, lib.cmpc_last_error().decode())
            self.instances.append(Problem(pr, _handle=h))

    def __len__(self):
        return self.count

    def __getitem__(self, i) -> Problem:
        return self.instances[i]

    def solve(self, **opts):
        """Returns (status, list of per-instance result dicts)."""
        o = default_options(**opts)
        res = (Result * self.count)()
        rc = load().cmpc_batch_solve(self._h, ctypes.byref(o), res)
        if rc < 0 and not any(r.status < 0 for r in res):
            _check(rc)
        return rc, [r.as_dict() for r in res]

    def solve_raw(self, options: Options, results) -> int:
        return load().cmpc_batch_solve(self._h, ctypes.byref(options), results)

    def solve_warm(self, v0s=None, **opts):
        """cmpc_batch_solve_warm: instance i starts from v0s[i] (float64 CUDA tensor, or None
        for its last solution shifted one stage); v0s None shifts every instance."""
        o = default_options(**opts)
        res = (Result * self.count)()
        if v0s is None:
            rc = load().cmpc_batch_solve_warm(self._h, ctypes.byref(o), None, 1, res)
        else:
            ptrs = (ctypes.c_void_p * self.count)(*[None if v is None else _dev(v) for v in v0s])
            rc = load().cmpc_batch_solve_warm(self._h, ctypes.byref(o), ptrs, 1, res)
        if rc < 0 and not any(r.status < 0 for r in res):
            _check(rc)
        return rc, [r.as_dict() for r in res]

    def tune(self, precision=FP64) -> dict:
        rep = TuneReport()
        _check(load().cmpc_batch_tune(self._h, precision, ctypes.byref(rep)))
        return rep.as_dict()

    def close(self):
        if self._h:
            for p in self.instances:
                p._h = ctypes.c_void_p()
            load().cmpc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hp(a):
    return ctypes.c_void_p(a.ctypes.data)


def default_train_opts(**kw) -> TrainOpts:
    o = TrainOpts()
    load().cmpc_default_train_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Mlp:
    """Surrogate policy x0 -> u for one problem (wraps cmpc_mlp).

    params: packed float32 initial parameters (W_1, b_1, ..., W_L+1, b_L+1).  Device inputs
    are float64 torch CUDA tensors: x0s (count x ns), ustars (count x nu N)."""

    def __init__(self, problem: Problem, params, hidden=1024, depth=4, precision=MLP_BF16):
        self.problem = problem          # the network answers this problem; keep it alive
        self.hidden, self.depth, self.precision = hidden, depth, precision
        p = np.ascontiguousarray(params, dtype=np.float32)
        w = [problem.ns] + [hidden] * depth + [problem.n]
        need = sum(w[l] * w[l - 1] + w[l] for l in range(1, len(w)))
        if p.size != need:
            raise ValueError(f"expected {need} packed parameters, got {p.size}")
        self._h = ctypes.c_void_p()
        _check(load().cmpc_mlp_create(problem._h, hidden, depth, precision, _hp(p),
                                      ctypes.byref(self._h)))
        self.nparams = int(load().cmpc_mlp_param_count(self._h))

    def close(self):
        if self._h:
            load().cmpc_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.empty(self.nparams, dtype=np.float32)
        _check(load().cmpc_mlp_get_params(self._h, _hp(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().cmpc_mlp_set_params(self._h, _hp(p)))

    def gradients(self, x0s, ustars):
        count = int(x0s.shape[0])
        g = np.empty(self.nparams, dtype=np.float32)
        loss = np.zeros(1)
        y = np.empty((count, self.problem.n), dtype=np.float32)
        _check(load().cmpc_mlp_gradients(self._h, _dev(x0s), _dev(ustars), count, _hp(g),
                                         _hp(loss), _hp(y)))
        return g, float(loss[0]), y

    def train(self, x0s, ustars, order=None, **opts):
        o = default_train_opts(**opts)
        count = int(x0s.shape[0])
        losses = np.zeros(o.epochs)
        ordp = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int32)
            assert order.size == o.epochs * count
            ordp = _hp(order)
        _check(load().cmpc_mlp_train(self._h, _dev(x0s), _dev(ustars), count, ctypes.byref(o),
                                     ordp, _hp(losses)))
        return losses

    def predict(self, x0s):
        import torch
        u = torch.empty((x0s.shape[0], self.problem.n), dtype=torch.float64, device=x0s.device)
        _check(load().cmpc_mlp_predict(self._h, _dev(x0s), int(x0s.shape[0]), _dev(u)))
        return u

    def judge(self, x0s, u):
        count = int(x0s.shape[0])
        acc = np.zeros(count, dtype=np.int32)
        vio, f, lb = np.zeros(count), np.zeros(count), np.zeros(count)
        _check(load().cmpc_judge(self._h, _dev(x0s), _dev(u), count, _hp(acc), _hp(vio), _hp(f),
                                 _hp(lb)))
        return acc.astype(bool), vio, f, lb

    def set_fallback(self, batch=None, warm=False):
        """Rejected answers are re-solved on `batch` (a Batch of copies of the network's
        problem, kept alive by this object) or one by one (None); warm: from the answer."""
        self._fallback = batch
        _check(load().cmpc_mlp_set_fallback(self._h, batch._h if batch is not None else None,
                                            1 if warm else 0))

    def solve(self, x0s):
        """(u device tensor, accepted bool array, report dict) for a batch of queries."""
        import torch
        count = int(x0s.shape[0])
        u = torch.empty((count, self.problem.n), dtype=torch.float64, device=x0s.device)
        acc = np.zeros(max(1, count), dtype=np.int32)
        rep = SurrogateReport()
        rc = load().cmpc_surrogate_solve(self._h, _dev(x0s), count, _dev(u), _hp(acc),
                                         ctypes.byref(rep))
        _check(rc, allow_positive=True)
        return u, acc[:count].astype(bool), rep.as_dict()


def tune_lookup(n, mx, precision=FP64):
    """(quantum, persistent) of the tuning-table entry, or None."""
    q, pers = ctypes.c_int(), ctypes.c_int()
    rc = load().cmpc_tune_lookup(n, mx, precision, ctypes.byref(q), ctypes.byref(pers))
    return (q.value, pers.value) if rc == 0 else None


def tune_store(n, mx, precision, quantum, persistent=1):
    """Record a tuning-table entry (SYRK work quantum and grid policy) for (n, mx, precision)."""
    _check(load().cmpc_tune_store(n, mx, precision, quantum, persistent))


def tune_clear():
    load().cmpc_tune_clear()


def potrf(K, ld=None):
    """In-place Cholesky of the lower triangle of a float64 CUDA tensor (n x ld)."""
    n = K.shape[0]
    info = ctypes.c_int(0)
    rc = load().cmpc_potrf(_dev(K), n, ld or K.shape[1], _stream(), ctypes.byref(info))
    _check(rc)
    return info.value


def potrf_noalloc(K, ld=None):
    """cmpc_potrf_noalloc: the same factorisation with the library's fixed device scratch
    (n <= POTRF_NOALLOC_MAX_N; allocates nothing)."""
    n = K.shape[0]
    info = ctypes.c_int(0)
    rc = load().cmpc_potrf_noalloc(_dev(K), n, ld or K.shape[1], _stream(), ctypes.byref(info))
    _check(rc)
    return info.value


def potrs(L, b, ld=None):
    n = L.shape[0]
    return _check(load().cmpc_potrs(_dev(L), n, ld or L.shape[1], _dev(b), _stream()))


def status_str(code: int) -> str:
    return load().cmpc_status_str(code).decode()
