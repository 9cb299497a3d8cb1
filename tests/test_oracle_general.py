"""Pins of the oracle's elimination for the general data of eqn. (sparse) -- the cross weight
S, the rows g^l <= E x + F u <= g^u, the disturbance w and the feedback u = K x + v of
eqn. (K_constraint) -- against checks written from eqn. (sparse) itself (``brute_force``):
forward simulation, the objective and every constraint evaluated on the simulated
trajectory, the cross-weight Riccati recursion, the invariance of the optimal inputs under
the choice of K, and exhaustive active-set enumeration of the sparse problem.  CPU only."""
from dataclasses import replace

import numpy as np
import pytest

import brute_force as bf
import oracle
from paper_2209_13049_amd import workloads as W

CASES = [  # (ns, nu, nc, N, seed, feedback, cross, w_scale)
    (3, 1, 1, 4, 0, True, True, 0.02),
    (4, 2, 2, 5, 1, True, True, 0.05),
    (5, 2, 0, 3, 2, False, True, 0.0),
    (4, 2, 1, 4, 3, True, False, 0.03),
    (2, 1, 2, 6, 4, False, False, 0.05),
]


def case(ns, nu, nc, N, seed, feedback, cross, w_scale, **kw):
    return W.general_random(ns, nu, nc, N, seed, feedback=feedback, cross=cross,
                            w_scale=w_scale, **kw)


@pytest.mark.parametrize("args", CASES)
def test_general_states_and_inputs_match_simulation(args):
    p = case(*args)
    red = oracle.reduce_problem(p)
    rng = np.random.default_rng(args[4])
    for _ in range(3):
        v = rng.normal(size=p.n)
        xs, us = bf.simulate_general(p, v)
        np.testing.assert_allclose(red.c + red.Gamma @ v, xs[1:].ravel(), rtol=1e-11,
                                   atol=1e-12)
        np.testing.assert_allclose(oracle.inputs(red, v), us.ravel(), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("args", CASES)
def test_general_objective_matches_sparse_objective(args):
    p = case(*args)
    red = oracle.reduce_problem(p)
    rng = np.random.default_rng(10 + args[4])
    for _ in range(3):
        v = rng.normal(size=p.n)
        xs, us = bf.simulate_general(p, v)
        f = bf.objective_general(p, xs, us)
        assert abs(oracle.objective(red, v) - f) <= 1e-11 * max(1.0, abs(f))


@pytest.mark.parametrize("args", CASES)
def test_general_rows_are_the_constraints(args):
    """J v - d, row by row, is the value of the inequality it encodes on the simulated
    trajectory (every kind of row, every stage)."""
    p = case(*args)
    red = oracle.reduce_problem(p)
    v = np.random.default_rng(20 + args[4]).normal(size=p.n)
    xs, us = bf.simulate_general(p, v)
    vals = bf.constraint_values(p, xs, us)
    got = red.J @ v - red.d
    assert sorted(set(red.groups)) == sorted(vals)
    for g, want in vals.items():
        np.testing.assert_allclose(got[red.groups == g], want[red.index[red.groups == g]],
                                   rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cross_weight_matches_riccati(seed):
    """No binding bound, no disturbance, no feedback: the minimiser is the LQR law with the
    cross weight S."""
    p = W.general_random(4, 2, 0, 6, seed, feedback=False, cross=True, w_scale=0.0, rho=0.9,
                         bound_x=1e3, bound_u=1e3)
    u_ric, f_ric = bf.riccati_cross(p)
    r = oracle.solve(p)
    assert r.status == oracle.STATUS_CONVERGED
    assert np.max(np.abs(r.u - u_ric)) <= 1e-7 * max(1.0, np.max(np.abs(u_ric)))
    assert abs(r.obj - f_ric) <= 1e-8 * max(1.0, abs(f_ric))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_optimal_inputs_do_not_depend_on_the_feedback(seed):
    """K only re-parametrises the inputs (u = K x + v): with and without it the problem in
    (x, u) is the same, so are its minimiser and optimal value."""
    with_k = W.general_random(4, 2, 1, 6, seed, feedback=True, rho=1.05)
    without = W.general_random(4, 2, 1, 6, seed, feedback=False, rho=1.05)
    assert with_k.Kfb is not None and without.Kfb is None
    a, b = oracle.solve(with_k), oracle.solve(without)
    assert a.status == b.status == oracle.STATUS_CONVERGED
    bound = max(1e-8, 2.0 * (a.gap + b.gap) / abs(b.obj))
    assert abs(a.obj - b.obj) <= bound * abs(b.obj)
    assert np.max(np.abs(a.u - b.u)) <= 1e-5


def tight_case(seed, fx, fu, fg):
    """A tiny instance (ns = 2, nu = 1, nc = 1, N = 2, with S, w and K) whose bounds are cut to
    the fractions fx, fu, fg of the largest |x_t|, |u_t|, |E x_t + F u_t| along its
    unconstrained optimum (found by the enumeration with no bound at all), so that they
    bind; x bounds never below |x0|."""
    p = W.general_random(2, 1, 1, 2, seed, feedback=True, bound_x=1e3, bound_u=1e3,
                         bound_g=1e3, w_scale=0.05, x0_scale=0.3)
    u_free, _ = bf.sparse_active_set(p)
    xs, us = bf.simulate_general(replace(p, Kfb=None), u_free)
    g = np.array([p.E @ xs[t] + p.F @ us[t] for t in range(p.N)])
    bx = max(1.01 * np.max(np.abs(p.x0)), fx * np.max(np.abs(xs[1:])))
    bu, bg = fu * np.max(np.abs(us)), fg * np.max(np.abs(g))
    return replace(p, xl=np.full(2, -bx), xu=np.full(2, bx), ul=np.full(1, -bu),
                   uu=np.full(1, bu), gl=np.full(1, -bg), gu=np.full(1, bg))


# feasible cut instances; together they bind state, input and general rows
TIGHT = [(3, 0.8, 0.8, 0.8), (3, 0.9, 0.7, 0.9), (4, 0.7, 0.9, 0.8), (10, 0.9, 0.7, 0.9)]


@pytest.mark.parametrize("args", TIGHT)
def test_general_matches_sparse_active_set(args):
    """The oracle's inputs and objective against the exact minimiser of eqn. (sparse)
    found by enumeration."""
    p = tight_case(*args)
    u_ex, f_ex = bf.sparse_active_set(p)
    r = oracle.solve(p)
    assert r.status == oracle.STATUS_CONVERGED
    assert abs(r.obj - f_ex) <= max(1e-8 * max(1.0, abs(f_ex)), 2.0 * r.gap)
    assert np.max(np.abs(r.u - u_ex)) <= 1e-5


def test_active_set_cases_bind_every_kind_of_row():
    """The enumeration cases are a check of every kind of row only if each kind binds."""
    kinds = set()
    for args in TIGHT:
        p = tight_case(*args)
        r = oracle.solve(p)
        red = oracle.reduce_problem(p)
        active = np.abs(red.J @ r.v - red.d) <= 1e-6
        kinds |= {int(g) // 2 for g in red.groups[active]}
    assert kinds == {0, 1, 2}, kinds


def test_heat_general_workload_binds_its_rows():
    """The GPU workload with general data: its stage rows bind at the optimum."""
    p = W.heat1d_general(40, 4, 10)
    r = oracle.solve(p)
    assert r.status == oracle.STATUS_CONVERGED
    red = oracle.reduce_problem(p)
    active = np.abs(red.J @ r.v - red.d) <= 1e-6
    assert np.any(np.isin(red.groups[active], [4, 5]))
    xs, us = bf.simulate_general(p, r.v)
    assert abs(bf.objective_general(p, xs, us) - r.obj) <= 1e-10 * max(1.0, abs(r.obj))
