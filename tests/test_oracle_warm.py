"""Pins of the oracle's receding-horizon loop and warm start (reading R14) against facts that
do not come from the oracle: a hand-worked shift, the start point's definition, the
uniqueness of the minimiser of the strictly convex QP (a warm start must not change it), and
the closed form of receding-horizon LQR (unconstrained: the first gain of the finite-horizon
Riccati recursion applied at every step).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import condensed_ipm as ipm
from paper_2209_13049_amd import workloads as W
from test_oracle_pins import random_stable


def test_shift_controls_hand_example():
    # nu = 2, N = 3: stages (1, 2), (3, 4), (5, 6) -> (3, 4), (5, 6), (5, 6)
    v = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    assert np.array_equal(ipm.shift_controls(v, 2, 3), [3.0, 4.0, 5.0, 6.0, 5.0, 6.0])
    # N = 1: the single stage is kept
    assert np.array_equal(ipm.shift_controls(np.array([7.0, 8.0]), 2, 1), [7.0, 8.0])


def test_warm_initial_point_definition():
    """From v0: s = max(d - J v0, 1e-2), lambda = z = mu0 / s (so r2 = 0); rows where
    d - J v0 >= 1e-2 start primal feasible (r3 = 0), the others with r3 = 1e-2 - (d - J v0)."""
    p = W.heat1d(30, 3, 8, seed=(0, 2), xu=0.05, x0_range=(-0.4, 0.04))
    red = oracle.reduce_problem(p)
    v0 = np.random.default_rng(5).uniform(-1.5, 1.5, p.n)
    v, s, lam, z = ipm.initial_point(red, 1e-3, v0)
    slack = red.d - red.J @ v0
    assert np.array_equal(v, v0)
    r3 = red.J @ v - red.d + s
    inside = slack >= 1e-2
    assert inside.any() and (~inside).any()
    assert np.all(np.abs(r3[inside]) <= 1e-15 * np.maximum(1.0, np.abs(red.d[inside])))
    assert np.allclose(r3[~inside], 1e-2 - slack[~inside], rtol=1e-12, atol=1e-15)
    assert np.allclose(lam * s, 1e-3, rtol=1e-15) and np.array_equal(lam, z)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_warm_start_reaches_the_same_minimiser(seed):
    """The QP is strictly convex (H >= Rbar > 0): from any start the method must converge to
    the one minimiser.  Warm starts from the shifted cold solution, from a random point and
    from the cold solution itself."""
    p = W.heat1d(40, 4, 12, seed=(seed, 1), xu=0.05, x0_range=(-0.4, 0.04))
    red = oracle.reduce_problem(p)
    cold = oracle.solve(p, red=red)
    starts = [ipm.shift_controls(cold.v, p.nu, p.N),
              np.random.default_rng(seed).uniform(-1.0, 1.0, p.n), cold.v]
    for v0 in starts:
        warm = oracle.solve(p, red=red, v0=v0)
        assert warm.status == cold.status == oracle.STATUS_CONVERGED
        bound = max(1e-8, 2.0 * (cold.gap + warm.gap) / abs(cold.obj))
        assert abs(warm.obj - cold.obj) <= bound * abs(cold.obj)
        assert np.max(np.abs(warm.v - cold.v)) <= 1e-4


@pytest.mark.parametrize("ns,nu,N,seed", [(4, 2, 6, 0), (6, 3, 5, 1)])
def test_closed_loop_unconstrained_is_receding_horizon_lqr(ns, nu, N, seed):
    """Bounds that never bind: every step applies u = -K_0 x with K_0 the first gain of the
    N-stage Riccati recursion (P_N = Q_f), so x_{k+1} = (A - B K_0) x_k; cold and warm loops
    alike."""
    p = random_stable(ns, nu, N, seed, bound_x=1e3, bound_u=1e3)
    P = p.Qf.copy()
    K = None
    for _ in range(N):
        K = np.linalg.solve(p.R + p.B.T @ P @ p.B, p.B.T @ P @ p.A)
        P = p.Q + p.A.T @ P @ (p.A - p.B @ K)
        P = 0.5 * (P + P.T)
    steps = 6
    x = p.x0.copy()
    ref = [x.copy()]
    for _ in range(steps):
        x = (p.A - p.B @ K) @ x
        ref.append(x.copy())
    ref = np.array(ref)
    for warm in (False, True):
        xs, us, results = ipm.closed_loop(p, steps, warm=warm)
        assert all(r.status == oracle.STATUS_CONVERGED for r in results)
        assert np.max(np.abs(xs - ref)) <= 1e-7 * max(1.0, np.max(np.abs(ref)))
        assert np.allclose(us[0], -K @ p.x0, rtol=1e-7, atol=1e-9)


def test_closed_loop_warm_equals_cold_trajectory():
    """With binding bounds the applied inputs do not depend on the start point (unique
    minimiser per step), and the warm loop takes fewer iterations after its first step."""
    p = W.heat1d(60, 4, 20, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    xs_c, us_c, rc = ipm.closed_loop(p, 4, warm=False)
    xs_w, us_w, rw = ipm.closed_loop(p, 4, warm=True)
    assert np.max(np.abs(us_w - us_c)) <= 1e-5
    assert np.max(np.abs(xs_w - xs_c)) <= 1e-6
    assert rw[0].iters == rc[0].iters
    assert sum(r.iters for r in rw[1:]) < sum(r.iters for r in rc[1:])
