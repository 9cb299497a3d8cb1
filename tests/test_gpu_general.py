"""General data of eqn. (sparse) on the GPU -- cross weight S, rows gl <= E x + F u <= gu,
disturbance w and the feedback u = K x + v of eqn. (K_constraint) -- against the oracle's
general elimination: FP64 takes the oracle's iteration count and reaches its objective,
inputs and states; the mixed modes meet the FP64 bar; a batch of such instances equals the
single solves bit for bit; data handed over in device memory give the same solve."""
import numpy as np
import pytest
import torch

import oracle
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu


def cases():
    out = {  # bounds chosen so that rows of each kind bind (checked against the oracle)
        "all": W.general_random(6, 2, 2, 8, 3, rho=1.05, bound_x=0.38, bound_u=0.5,
                                bound_g=0.12),
        "all_upper": W.general_random(6, 2, 2, 8, 0, rho=1.05, bound_x=0.38, bound_u=0.5,
                                      bound_g=0.12),
        "feedback_only": W.general_random(5, 2, 0, 7, 1, cross=False, w_scale=0.0, rho=1.1,
                                          bound_x=0.35, bound_u=0.4),
        "rows_only": W.general_random(6, 3, 3, 6, 2, feedback=False, cross=False,
                                      w_scale=0.0, rho=0.9, bound_g=0.15),
        "cross_w": W.general_random(7, 2, 0, 9, 1, feedback=False, rho=0.95, bound_x=0.25,
                                    bound_u=0.4, x0_scale=0.2),
        "heat": W.heat1d_general(40, 4, 10),
        "heat_tiles": W.heat1d_general(90, 9, 16, kgain=0.3),   # K 144 x 144: three tiles
    }
    return out


CASES = cases()


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / max(1.0, float(np.max(np.abs(b))))


@pytest.fixture(scope="module")
def refs():
    return {k: oracle.solve(p) for k, p in CASES.items()}


def check(tag, res, ref, u, x, iters_equal=True):
    print(f"[general] {tag}: gpu iters {res['iters']} obj {res['obj']:.12e} | oracle iters "
          f"{ref.iters} obj {ref.obj:.12e}", flush=True)
    assert res["status"] == condmpc.OK and ref.status == oracle.STATUS_CONVERGED
    if iters_equal:
        assert res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
    assert rel_err(u, ref.u) <= 1e-6
    assert rel_err(x, ref.x) <= 1e-6


@pytest.mark.parametrize("name", sorted(CASES))
def test_general_fp64_matches_oracle(lib, refs, name):
    p = CASES[name]
    gp = condmpc.Problem(p)
    try:
        gp.set_x0(p.x0)
        res = gp.solve()
        u, x = gp.solution()
        check(name, res, refs[name], u, x)
    finally:
        gp.close()


@pytest.mark.parametrize("name", ["heat", "heat_tiles", "all"])
def test_general_mixed_precision(lib, refs, name):
    p = CASES[name]
    gp = condmpc.Problem(p)
    try:
        gp.set_x0(p.x0)
        for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            res = gp.solve(precision=prec)
            u, x = gp.solution()
            check(f"{name} prec {prec}", res, refs[name], u, x, iters_equal=False)
    finally:
        gp.close()


def test_general_batch_equals_single(lib, refs):
    names = sorted(CASES)
    probs = [CASES[k] for k in names]
    b = condmpc.Batch(probs)
    try:
        rc, results = b.solve()
        assert rc == condmpc.OK
        for i, k in enumerate(names):
            ub, xb = b[i].solution()
            check(f"batch {k}", results[i], refs[k], ub, xb)
            single = condmpc.Problem(probs[i])
            single.set_x0(probs[i].x0)
            r = single.solve()
            us, xs = single.solution()
            single.close()
            assert r["iters"] == results[i]["iters"] and np.array_equal(us, ub), k
    finally:
        b.close()


def test_general_data_on_device(lib, refs):
    p = CASES["all"]
    host = condmpc.Problem(p)
    dev = condmpc.Problem(p, device_data=True)
    try:
        host.set_x0(p.x0)
        dev.set_x0(p.x0)
        rh, rd = host.solve(), dev.solve()
        uh, _ = host.solution(with_x=False)
        ud, _ = dev.solution(with_x=False)
        assert rh["iters"] == rd["iters"] and np.array_equal(uh, ud)
    finally:
        host.close()
        dev.close()


def test_general_invalid_data(lib):
    from dataclasses import replace
    p = CASES["rows_only"]
    bad = replace(p, gl=p.gu + 0.1)
    with pytest.raises(condmpc.CmpcError) as e:
        condmpc.Problem(bad)
    assert e.value.code == condmpc.ERR_INVALID
    nanS = replace(CASES["cross_w"], S=np.full_like(CASES["cross_w"].S, np.nan))
    with pytest.raises(condmpc.CmpcError) as e:
        condmpc.Problem(nanS)
    assert e.value.code == condmpc.ERR_NONFINITE
