"""Degenerate shapes and data on the GPU against the oracle: a horizon of one stage (K 1 x 1 and
K 3 x 3), a scalar system over six stages, every bound infinite (no inequality row can bind, so
Algorithm 1 ends after one Newton step on the quadratic), and an initial state lying on its
bounds.  Same iteration counts, objectives within 1e-8, inputs within 1e-6; the mixed modes
meet the FP64 bar.  The CPU test below checks that the bounded cases really bind."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from paper_2209_13049_amd import condmpc
from test_oracle_pins import random_stable


def cases():
    out = {
        "scalar_N1": random_stable(1, 1, 1, 11, bound_u=0.001, bound_x=0.5, x0_scale=0.45),
        "ns1_N6": random_stable(1, 1, 6, 12, bound_u=0.01, bound_x=0.3, x0_scale=0.29),
        "nu1_N1": random_stable(4, 1, 1, 13, bound_u=0.005),
        "N1_nu3": random_stable(5, 3, 1, 14, bound_u=0.005),
    }
    p = random_stable(4, 2, 5, 15)
    inf, infu = np.full(p.ns, np.inf), np.full(p.nu, np.inf)
    out["unbounded"] = replace(p, xl=-inf, xu=inf, ul=-infu, uu=infu)
    q = random_stable(3, 2, 6, 16, x0_scale=0.5, bound_x=0.5)
    x0 = q.x0.copy()
    x0[0], x0[1] = 0.5, -0.5  # on the upper and the lower state bound
    out["x0_on_bound"] = replace(q, x0=x0)
    return out


CASES = cases()
BINDING = ["scalar_N1", "ns1_N6", "nu1_N1", "N1_nu3", "x0_on_bound"]


def test_bounded_cases_bind():
    """CPU: at the oracle's optimum at least one inequality row of each bounded case is active,
    and the unbounded case keeps no row at all."""
    for name in BINDING:
        p = CASES[name]
        r = oracle.solve(p)
        red = oracle.reduce_problem(p)
        assert r.status == oracle.STATUS_CONVERGED
        assert np.sum(np.abs(red.J @ r.v - red.d) <= 1e-6) >= 1, name
    assert oracle.reduce_problem(CASES["unbounded"]).J.shape[0] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_matches_oracle(lib, name):
    p = CASES[name]
    ref = oracle.solve(p)
    gp = condmpc.Problem(p)
    try:
        gp.set_x0(p.x0)
        res = gp.solve()
        u, x = gp.solution()
        print(f"[degenerate] {name}: gpu iters {res['iters']} obj {res['obj']:.12e} | oracle "
              f"iters {ref.iters} obj {ref.obj:.12e}", flush=True)
        assert res["status"] == condmpc.OK and ref.status == oracle.STATUS_CONVERGED
        assert res["iters"] == ref.iters
        assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
        assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
        assert np.max(np.abs(u - ref.v)) <= 1e-6 * max(1.0, np.max(np.abs(ref.v)))
        assert np.max(np.abs(x - oracle.simulate(p, u))) <= 1e-12 * max(1.0, np.max(np.abs(x)))
        for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            r = gp.solve(precision=prec)
            assert r["status"] == condmpc.OK
            assert abs(r["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    finally:
        gp.close()
