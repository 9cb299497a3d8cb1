"""Warm starts and the receding-horizon loop on the GPU (cmpc_solve_warm) against the
oracle's reading R14: from given controls, and from the previous step's controls shifted one
stage (the controller of Section 1, which solves again from each new state and applies the
first input).  FP64 takes the oracle's iteration counts; the mixed modes meet the FP64 bar."""
import numpy as np
import pytest

import oracle
from oracle import condensed_ipm as ipm
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / max(1.0, float(np.max(np.abs(b))))


def check(res, ref, u, iters_equal=True):
    assert res["status"] == condmpc.OK and ref.status == oracle.STATUS_CONVERGED
    if iters_equal:
        assert res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
    assert rel_err(u, ref.v) <= 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_warm_start_from_given_controls(lib, seed):
    p = W.heat1d(40, 4, 12, seed=(seed, 1), xu=0.05, x0_range=(-0.4, 0.04))
    red = oracle.reduce_problem(p)
    v0 = np.random.default_rng(seed).uniform(-1.0, 1.0, p.n)
    ref = oracle.solve(p, red=red, v0=v0)
    gp = condmpc.Problem(p)
    try:
        gp.set_x0(p.x0)
        res = gp.solve_warm(v0)
        u, _ = gp.solution(with_x=False)
        print(f"[warm] seed {seed}: gpu iters {res['iters']} oracle {ref.iters}", flush=True)
        check(res, ref, u)
        for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            res = gp.solve_warm(v0, precision=prec)
            u, _ = gp.solution(with_x=False)
            check(res, ref, u, iters_equal=False)
    finally:
        gp.close()


def test_receding_horizon_loop_matches_oracle(lib):
    """Four receding-horizon steps with binding state bounds: cold first solve, then warm
    starts from the shifted controls after each new state x+ = A x + B u_0."""
    p = W.heat1d(60, 4, 20, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    steps = 4
    xs_ref, us_ref, results = ipm.closed_loop(p, steps, warm=True)
    gp = condmpc.Problem(p)
    try:
        x = p.x0.copy()
        for k in range(steps):
            gp.set_x0(x)
            res = gp.solve() if k == 0 else gp.solve_warm()
            u, _ = gp.solution(with_x=False)
            print(f"[loop] step {k}: gpu iters {res['iters']} oracle {results[k].iters}",
                  flush=True)
            check(res, results[k], u)
            u0 = u[:p.nu]
            assert np.max(np.abs(u0 - us_ref[k])) <= 1e-6
            x = p.A @ x + p.B @ u0
            assert np.max(np.abs(x - xs_ref[k + 1])) <= 1e-6
        assert sum(r.iters for r in results[1:]) < (steps - 1) * results[0].iters
    finally:
        gp.close()


def test_warm_without_previous_solve_is_an_error(lib):
    p = W.heat1d(20, 2, 5, seed=(0, 4))
    gp = condmpc.Problem(p)
    try:
        gp.set_x0(p.x0)
        with pytest.raises(condmpc.CmpcError) as e:
            gp.solve_warm()
        assert e.value.code == condmpc.ERR_INVALID
        with pytest.raises(condmpc.CmpcError) as e:
            gp.solve_warm(np.zeros(p.n), warm_mu=0.0)
        assert e.value.code == condmpc.ERR_INVALID
        with pytest.raises(condmpc.CmpcError) as e:
            gp.solve_warm(np.full(p.n, np.nan))
        assert e.value.code == condmpc.ERR_NONFINITE
    finally:
        gp.close()
