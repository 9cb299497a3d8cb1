"""Pins of the oracle's barrier-parameter rule (reading R8) against hand-worked values.

Algorithm 1 of the paper leaves the update of mu open; the oracle takes the monotone rule of
Waechter and Biegler's IPOPT paper.  tests/golden/mu_rule.json holds rule applications
worked by hand (each one turns on one constant or one term of E_mu) and the first three
barrier values of a one-row scalar problem, derived by hand through three Newton steps.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2209_13049_amd.workloads import LQProblem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mu_rule.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _arr(x):
    return np.asarray(x, dtype=np.float64)


def rule_case_errors(mod):
    """Names of the golden rule cases `mod.barrier_update` gets wrong."""
    bad = []
    for c in _golden()["rule_cases"]:
        mu, tau = mod.barrier_update(c["mu"], _arr(c["r1"]), _arr(c["r3"]), _arr(c["lam"]),
                                     _arr(c["z"]), _arr(c["s"]), c["tol"] / 10.0)
        if abs(mu - c["mu_new"]) > 1e-12 * c["mu_new"] or abs(tau - c["tau"]) > 1e-14:
            bad.append((c["name"], mu, tau))
    return bad


def scalar_problem():
    g = _golden()["scalar_sequence"]["problem"]
    one = lambda v: np.array([[float(v)]])
    vec = lambda v: np.array([float(v)])
    return LQProblem(A=one(g["A"]), B=one(g["B"]), Q=one(g["Q"]), R=one(g["R"]),
                     Qf=one(g["Qf"]), xl=vec(g["xl"]), xu=vec(g["xu"]), ul=vec(g["ul"]),
                     uu=vec(g["uu"]), x0=vec(g["x0"]), N=int(g["N"]), name="scalar_one_row")


def scalar_mu_sequence(mod):
    r = mod.solve(scalar_problem(), tol=_golden()["scalar_sequence"]["problem"]["tol"],
                  record=True)
    return [h["mu"] for h in r.history[:3]], r


@pytest.mark.parametrize("case", _golden()["rule_cases"], ids=lambda c: c["name"])
def test_rule_case(case):
    mu, tau = oracle.condensed_ipm.barrier_update(
        case["mu"], _arr(case["r1"]), _arr(case["r3"]), _arr(case["lam"]), _arr(case["z"]),
        _arr(case["s"]), case["tol"] / 10.0)
    assert mu == pytest.approx(case["mu_new"], rel=1e-12, abs=0)
    assert tau == pytest.approx(case["tau"], rel=0, abs=1e-14)


def test_scalar_first_three_mu():
    want = _golden()["scalar_sequence"]["mu"]
    got, r = scalar_mu_sequence(oracle.condensed_ipm)
    assert len(got) == 3
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
    # and the problem itself: the optimum of 1/2 (u^2 + u^2) with u <= 1 is u = 0
    assert r.status == 0 and abs(r.v[0]) <= 1e-8 and abs(r.obj) <= 1e-8


def test_solve_uses_the_rule_every_iteration():
    """Every recorded mu is reached from the previous one by the rule: either it is the
    previous one, or the previous one mapped k >= 1 times by max(mu_min, min(0.2 mu,
    mu^1.5)) (the orbit is computed here by hand-entered constants)."""
    from paper_2209_13049_amd import workloads as W
    p = W.heat1d(30, 3, 6, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    tol = 1e-8
    r = oracle.solve(p, tol=tol, record=True)
    assert r.status == 0
    mus = [0.1] + [h["mu"] for h in r.history]
    for a, b in zip(mus[:-1], mus[1:]):
        orbit, x = [a], a
        while x > tol / 10:
            x = max(tol / 10, min(0.2 * x, x ** 1.5))
            orbit.append(x)
        assert any(b == o for o in orbit), (a, b)
