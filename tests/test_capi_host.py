"""Host-side checks of the C ABI (no GPU needed): the shared library loads and exports every
function that include/condmpc.h declares, and the binding's structures match the header."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2209_13049_amd import condmpc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "condmpc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmpc_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(condmpc.EXPORTS)


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(condmpc.LIB_PATH):
        from paper_2209_13049_amd import build
        build.build()
    return condmpc.LIB_PATH


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\b(cmpc_[a-z0-9_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, f"not exported: {missing}"


def test_library_loads_and_binds(built):
    lib = condmpc.load()
    for name in condmpc.EXPORTS:
        assert hasattr(lib, name)
    # pure host functions can be called without a GPU
    o = condmpc.default_options()
    assert o.tol == 1e-8 and o.max_iter == 200 and o.precision == condmpc.FP64
    assert o.check_every == 2 and o.profile == 0 and o.equilibrate == -1
    assert condmpc.status_str(condmpc.ERR_CHOLESKY) == "Cholesky breakdown"
    assert condmpc.status_str(condmpc.OK) == "converged"


def test_struct_layouts_match_header():
    text = open(HEADER).read()

    def fields(struct_name):
        m = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct_name + ";", text)
        body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            fp = re.match(r"[^(]*\(\*\s*([A-Za-z_][A-Za-z0-9_]*)\s*\)", decl)
            if fp:  # function pointer: void (*name)(args)
                names.append(fp.group(1))
                continue
            for part in decl.split(","):
                names.append(re.findall(r"[A-Za-z_][A-Za-z0-9_]*", part)[-1])
        return names

    assert fields("cmpc_lq_desc") == [f for f, _ in condmpc.LQDesc._fields_]
    assert fields("cmpc_options") == [f for f, _ in condmpc.Options._fields_]
    assert fields("cmpc_result") == [f for f, _ in condmpc.Result._fields_]
    assert fields("cmpc_info") == [f for f, _ in condmpc.Info._fields_]
    assert fields("cmpc_tune_report") == [f for f, _ in condmpc.TuneReport._fields_]
    assert fields("cmpc_train_opts") == [f for f, _ in condmpc.TrainOpts._fields_]
    assert fields("cmpc_surrogate_report") == [f for f, _ in condmpc.SurrogateReport._fields_]


def test_null_arguments_are_rejected_without_gpu(built):
    lib = condmpc.load()
    assert lib.cmpc_problem_create(None, None, None) == condmpc.ERR_INVALID
    assert lib.cmpc_solve(None, None, None) == condmpc.ERR_INVALID
    assert lib.cmpc_problem_dims(None, None, None, None) == condmpc.ERR_INVALID
    assert b"NULL" in lib.cmpc_last_error()


def _desc(ns=3, nu=2, N=4, **over):
    import numpy as np
    rng = np.random.default_rng(0)
    arrs = dict(A=0.5 * np.eye(ns), B=rng.normal(size=(ns, nu)), Q=np.eye(ns), R=np.eye(nu),
                Qf=np.eye(ns), xl=-np.ones(ns), xu=np.ones(ns), ul=-np.ones(nu), uu=np.ones(nu))
    arrs.update(over)
    keep = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in arrs.items()}
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d = condmpc.LQDesc(ns=ns, nu=nu, N=N, **{k: P(v) for k, v in keep.items()})
    return d, keep


@pytest.mark.parametrize("case,code", [
    ("nan_A", condmpc.ERR_NONFINITE), ("R_not_pd", condmpc.ERR_INVALID),
    ("R_not_symmetric", condmpc.ERR_INVALID), ("bad_u_bounds", condmpc.ERR_INVALID),
    ("bad_x_bounds", condmpc.ERR_INVALID), ("nan_bound", condmpc.ERR_NONFINITE),
    ("zero_horizon", condmpc.ERR_INVALID)])
def test_invalid_problem_data_rejected_on_host(built, case, code):
    """Validation happens before any device work, so these run without a GPU."""
    import numpy as np
    over, N = {}, 4
    if case == "nan_A":
        A = 0.5 * np.eye(3); A[1, 2] = np.nan; over["A"] = A
    elif case == "R_not_pd":
        over["R"] = np.array([[1.0, 2.0], [2.0, 1.0]])
    elif case == "R_not_symmetric":
        over["R"] = np.array([[1.0, 0.5], [0.0, 1.0]])
    elif case == "bad_u_bounds":
        over["ul"] = np.array([1.0, -1.0])
    elif case == "bad_x_bounds":
        over["xl"] = np.array([2.0, -1.0, -1.0])
    elif case == "nan_bound":
        over["xu"] = np.array([np.nan, 1.0, 1.0])
    elif case == "zero_horizon":
        N = 0
    d, keep = _desc(N=N, **over)
    h = ctypes.c_void_p()
    rc = condmpc.load().cmpc_problem_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == code, condmpc.load().cmpc_last_error()
    assert not h.value


def test_batch_calls_without_gpu(built):
    lib = condmpc.load()
    h = ctypes.c_void_p()
    assert lib.cmpc_batch_create(0, None, None, None, ctypes.byref(h)) == condmpc.ERR_INVALID
    assert not h.value
    assert lib.cmpc_batch_size(None) == 0
    assert lib.cmpc_batch_instance(None, 0) is None
    assert lib.cmpc_batch_solve(None, None, None) == condmpc.ERR_INVALID
    assert lib.cmpc_batch_tune(None, condmpc.FP64, None) == condmpc.ERR_INVALID
    lib.cmpc_tune_clear()
    assert lib.cmpc_tune_lookup(64, 100, condmpc.FP64, None, None) == 1
    assert condmpc.tune_lookup(64, 100) is None


def test_batch_rejects_invalid_instance_on_host(built):
    """Validation of the first instance happens before any device work."""
    import numpy as np
    A = 0.5 * np.eye(3)
    A[0, 1] = np.inf
    d, keep = _desc(A=A)
    descs = (condmpc.LQDesc * 2)(d, d)
    h = ctypes.c_void_p()
    rc = condmpc.load().cmpc_batch_create(2, descs, None, None, ctypes.byref(h))
    assert rc == condmpc.ERR_NONFINITE
    assert b"instance 0" in condmpc.load().cmpc_last_error()
    assert not h.value


def test_surrogate_calls_without_gpu(built):
    lib = condmpc.load()
    o = condmpc.default_train_opts()
    assert o.batch == 512 and o.epochs == 20 and abs(o.lr - 1e-3) < 1e-9
    h = ctypes.c_void_p()
    assert lib.cmpc_mlp_create(None, 64, 2, condmpc.MLP_BF16, None, ctypes.byref(h)) == \
        condmpc.ERR_INVALID
    assert lib.cmpc_mlp_param_count(None) == 0
    assert lib.cmpc_mlp_train(None, None, None, 0, None, None, None) == condmpc.ERR_INVALID
    assert lib.cmpc_surrogate_solve(None, None, 0, None, None, None) == condmpc.ERR_INVALID
