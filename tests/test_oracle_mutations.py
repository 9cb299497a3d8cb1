"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each case edits one expression of ``oracle/condensed_ipm.py`` in memory (a dropped term, a
wrong sign, an off-by-one power, a transposed operand, a wrong constant), loads the edited
source as a separate module and runs the independent checks of ``test_oracle_pins`` against
it.  At least one check must fail for every mutant; the unedited source passes them all.
"""
import os
import sys
import types

import numpy as np
import pytest

import brute_force as bf
import test_oracle_barrier as tb
import test_oracle_general as tg
from paper_2209_13049_amd import workloads as W
from test_oracle_pins import random_stable, _binding_case, _pairs, _interior_point

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "condensed_ipm.py")

MUTATIONS = {
    "gamma_power_off_by_one": ("Gamma[(t - 1) * ns:t * ns, j * nu:(j + 1) * nu] = G[t - 1 - j]",
                               "Gamma[(t - 1) * ns:t * ns, j * nu:(j + 1) * nu] = G[max(t - 2 - j, 0)]"),
    "gamma_transposed_power": ("out.append(A @ out[-1])", "out.append(A.T @ out[-1])"),
    "terminal_weight_dropped": ("W = Qf if t == N else Q", "W = Q"),
    "h0_half_dropped": ("h0 = 0.5 * prob.x0 @ Q @ prob.x0 + 0.5 * c @ qbar_times(c)",
                        "h0 = 0.5 * c @ qbar_times(c)"),
    "rhs_sigma_r3_sign": ("rhs = -r1 + red.J.T @ r2 - red.J.T @ (sigma * r3)",
                          "rhs = -r1 + red.J.T @ r2 + red.J.T @ (sigma * r3)"),
    "rhs_r2_dropped": ("rhs = -r1 + red.J.T @ r2 - red.J.T @ (sigma * r3)",
                       "rhs = -r1 - red.J.T @ (sigma * r3)"),
    "plam_sigma_r3_dropped": ("plam = -r2 + sigma * r3 + sigma * Jpv", "plam = -r2 + sigma * Jpv"),
    "pz_sign": ("pz = mu / s - z - sigma * ps", "pz = mu / s - z + sigma * ps"),
    "ps_sign": ("ps = -r3 - Jpv", "ps = -r3 + Jpv"),
    "sigma_inverted": ("sigma = z / s\n    r1, r2, r3", "sigma = s / z\n    r1, r2, r3"),
    "ftb_no_tau": ("return float(min(1.0, np.min(-tau * x[neg] / p[neg])))",
                   "return float(min(1.0, np.min(-x[neg] / p[neg])))"),
    "lower_state_rows_sign": ("d_all = np.concatenate([xu - c, c - xl, uu, -ul])",
                              "d_all = np.concatenate([xu - c, c + xl, uu, -ul])"),
    "r1_lambda_dropped": ("r1 = red.H @ v + red.h + red.J.T @ lam\n    r2",
                          "r1 = red.H @ v + red.h\n    r2"),
    "alpha_z_for_lambda": ("lam = lam + alpha * step[\"plam\"]", "lam = lam + alpha_z * step[\"plam\"]"),
    # the barrier rule (reading R8) and its error measure
    "kappa_eps_1": ("KAPPA_EPS = 10.0", "KAPPA_EPS = 1.0"),
    "kappa_mu_half": ("KAPPA_MU = 0.2", "KAPPA_MU = 0.5"),
    "theta_mu_2": ("THETA_MU = 1.5", "THETA_MU = 2.0"),
    "mu_rule_max_for_min": ("mu = max(mu_min, min(KAPPA_MU * mu, mu ** THETA_MU))",
                            "mu = max(mu_min, max(KAPPA_MU * mu, mu ** THETA_MU))"),
    "mu_floor_tol": ("mu_min = tol / 10.0", "mu_min = tol"),
    "tau_fixed": ("return mu, max(TAU_MIN, 1.0 - mu)", "return mu, TAU_MIN"),
    "tau_min_for_max": ("return mu, max(TAU_MIN, 1.0 - mu)", "return mu, min(TAU_MIN, 1.0 - mu)"),
    "emu_lambda_z_dropped": ("np.max(np.abs(lam - z), initial=0.0), np.max(np.abs(s * z - mu)",
                             "0.0, np.max(np.abs(s * z - mu)"),
    "emu_r3_dropped": ("parts = [np.max(np.abs(r1), initial=0.0), np.max(np.abs(r3), initial=0.0),",
                       "parts = [np.max(np.abs(r1), initial=0.0), 0.0,"),
    "emu_complementarity_not_shifted": ("np.max(np.abs(s * z - mu), initial=0.0)]",
                                        "np.max(np.abs(s * z), initial=0.0)]"),
    "emu_stationarity_dropped": ("parts = [np.max(np.abs(r1), initial=0.0),",
                                 "parts = [0.0,"),
    # the receding-horizon warm start (reading R14)
    "shift_wrong_direction": ("return np.concatenate([v[nu:nu * N], v[nu * (N - 1):nu * N]])",
                              "return np.concatenate([v[:nu], v[:nu * (N - 1)]])"),
    "shift_last_stage_zero": ("return np.concatenate([v[nu:nu * N], v[nu * (N - 1):nu * N]])",
                              "return np.concatenate([v[nu:nu * N], 0.0 * v[:nu]])"),
    "warm_start_ignored": ("v = np.zeros(n) if v0 is None else np.array(v0, dtype=np.float64)",
                           "v = np.zeros(n)"),
    "warm_mu_cold_value": ("WARM_MU_INIT = 1e-3\nS_INIT_MIN", "WARM_MU_INIT = 0.1\nS_INIT_MIN"),
    "closed_loop_last_input": ("u0 = r.v[:nu].copy()", "u0 = r.v[-nu:].copy()"),
    "closed_loop_no_input": ("x = prob.A @ x + prob.B @ u0", "x = prob.A @ x"),
    # the elimination with general data (S, E/F rows, w, feedback K)
    "general_w_dropped": ("X0.append(AK @ X0[t] + w[t])", "X0.append(AK @ X0[t])"),
    "general_open_loop_powers": ("AK = A + B @ K", "AK = A"),
    "general_feedback_dropped_from_inputs": ("UV.append(K @ XV[t] + sel)", "UV.append(sel)"),
    "general_cross_half_dropped": ("Wst = np.block([[Q, S], [S.T, R]])",
                                   "Wst = np.block([[Q, 0.0 * S], [S.T, R]])"),
    "general_terminal_weight_Q": ("Wbar = sla.block_diag(*([Wst] * N + [Qf]))",
                                  "Wbar = sla.block_diag(*([Wst] * N + [Q]))"),
    "general_F_dropped": ("Cv = np.vstack([E @ XV[t] + F @ UV[t] for t in range(N)])",
                          "Cv = np.vstack([E @ XV[t] for t in range(N)])"),
    "general_g_lower_sign": ("(-Cv, c0 - np.tile(prob.gl, N), 5)",
                             "(-Cv, c0 + np.tile(prob.gl, N), 5)"),
    "general_input_lower_sign": ("(-Uv, u0 - np.tile(prob.ul, N), 3)",
                                 "(-Uv, u0 + np.tile(prob.ul, N), 3)"),
    "general_stage_offset": ("sel[:, t * nu:(t + 1) * nu] = np.eye(nu)",
                             "sel[:, max(t - 1, 0) * nu:max(t, 1) * nu] = np.eye(nu)"),
}


def load_variant(name=None):
    src = open(SRC).read()
    if name is not None:
        old, new = MUTATIONS[name]
        assert src.count(old) >= 1, f"mutation anchor for {name} not found"
        src = src.replace(old, new, 1)
    mod = types.ModuleType(f"oracle_variant_{name}")
    sys.modules[mod.__name__] = mod        # dataclasses look their module up here
    exec(compile(src, SRC, "exec"), mod.__dict__)
    return mod


def check_simulation(m):
    p = random_stable(4, 2, 4, 1)
    red = m.reduce_problem(p)
    v = np.random.default_rng(0).normal(size=p.n)
    np.testing.assert_allclose(red.c + red.Gamma @ v, m.simulate(p, v), rtol=1e-12, atol=1e-12)


def check_objective(m):
    p = random_stable(3, 2, 3, 2)
    red = m.reduce_problem(p)
    v = np.random.default_rng(1).normal(size=p.n)
    assert abs(m.objective(red, v) - m.sparse_objective(p, v)) <= 1e-12 * 10


def check_full_space(m):
    p = random_stable(3, 1, 3, 1)
    red = m.reduce_problem(p)
    v, s, lam, z, mu = _interior_point(red, 1)
    st = m.condensed_step(red, v, s, lam, z, mu)
    pu, ps, plam, pz = bf.full_space_step(p, v, s, lam, z, mu)
    np.testing.assert_allclose(st["pv"], pu, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(st["ps"], ps, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(st["plam"], plam, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(st["pz"], pz, rtol=1e-9, atol=1e-9)


def check_ftb(m):
    s = np.array([1.0, 2.0, 0.5, 3.0])
    p = np.array([-2.0, 1.0, -0.1, -0.5])
    assert abs(m.fraction_to_boundary(s, p, 0.99) - 0.495) <= 1e-15


def check_riccati(m):
    p = random_stable(4, 2, 6, 1, bound_x=1e3, bound_u=1e3)
    r = m.solve(p, max_iter=60)
    u_ric, f_ric = bf.riccati(p)
    assert r.status == 0
    assert np.max(np.abs(r.v - u_ric)) <= 1e-7 * max(1.0, np.max(np.abs(u_ric)))


def check_active_set(m):
    for seed, kind in ((40, "u"), (40, "x")):
        p = _binding_case(seed, kind)
        red = m.reduce_problem(p)
        r = m.solve(p, max_iter=60)
        assert r.status == 0
        v_ex, _ = bf.active_set(red.H, red.h, red.J, red.d, _pairs(red, 2, 1, 3))
        f_ex = m.objective(red, v_ex)
        assert r.obj >= f_ex - 1e-12 and r.obj - f_ex <= r.gap + 1e-12


def check_tight_converges(m):
    p = W.heat1d(30, 3, 6, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    r = m.solve(p, max_iter=60)
    assert r.status == 0 and r.primal_res <= 1e-8 and r.dual_res <= 1e-8


def check_linear_residual_decay(m):
    """r1 and r3 are affine in (v, lambda, s): a step of length alpha shrinks both by
    exactly (1 - alpha)."""
    p = W.heat1d(20, 2, 5, seed=(5, 0), xu=0.05, x0_range=(0.045, 0.05))
    log = []
    m.solve(p, callback=log.append, max_iter=60)
    for a, b in zip(log[:-1], log[1:]):
        np.testing.assert_allclose(b["r3"], (1 - a["alpha"]) * a["r3"], atol=1e-12)
        np.testing.assert_allclose(b["r1"], (1 - a["alpha"]) * a["r1"], atol=1e-10)


def check_barrier_rule(m):
    bad = tb.rule_case_errors(m)
    assert not bad, bad


def check_scalar_mu_sequence(m):
    got, _ = tb.scalar_mu_sequence(m)
    np.testing.assert_allclose(got, tb._golden()["scalar_sequence"]["mu"], rtol=1e-12, atol=0)


def check_shift(m):
    v = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    assert np.array_equal(m.shift_controls(v, 2, 3), [3.0, 4.0, 5.0, 6.0, 5.0, 6.0])


def check_warm_start_point(m):
    """The start point from given controls (reading R14): r3 = 0 on rows with slack >= 1e-2,
    lambda s = 1e-3, and the first barrier parameter of a start far from the solution is
    that value."""
    p = W.heat1d(20, 2, 6, seed=(0, 2), xu=0.05, x0_range=(-0.4, 0.04))
    red = m.reduce_problem(p)
    v0 = np.random.default_rng(5).uniform(-1.5, 1.5, p.n)
    r = m.solve(p, red=red, v0=v0, record=True, max_iter=1)
    assert r.history[0]["mu"] == 1e-3
    v, s, lam, z = m.initial_point(red, 1e-3, v0)
    slack = red.d - red.J @ v0
    inside = slack >= 1e-2
    r3 = red.J @ v - red.d + s
    np.testing.assert_allclose(r3[inside], 0.0, atol=1e-14)
    np.testing.assert_allclose(r3[~inside], 1e-2 - slack[~inside], rtol=1e-12)


def check_closed_loop_lqr(m):
    p = random_stable(4, 2, 6, 0, bound_x=1e3, bound_u=1e3)
    P, K = p.Qf.copy(), None
    for _ in range(p.N):
        K = np.linalg.solve(p.R + p.B.T @ P @ p.B, p.B.T @ P @ p.A)
        P = p.Q + p.A.T @ P @ (p.A - p.B @ K)
    xs, us, _ = m.closed_loop(p, 3, warm=True)
    x = p.x0.copy()
    for k in range(3):
        x = (p.A - p.B @ K) @ x
        assert np.max(np.abs(xs[k + 1] - x)) <= 1e-7


def check_general_simulation(m):
    for args in tg.CASES[:2]:
        p = tg.case(*args)
        red = m.reduce_problem(p)
        v = np.random.default_rng(3).normal(size=p.n)
        xs, us = bf.simulate_general(p, v)
        np.testing.assert_allclose(red.c + red.Gamma @ v, xs[1:].ravel(), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(m.inputs(red, v), us.ravel(), rtol=1e-11, atol=1e-12)


def check_general_objective(m):
    p = tg.case(*tg.CASES[0])
    red = m.reduce_problem(p)
    v = np.random.default_rng(4).normal(size=p.n)
    xs, us = bf.simulate_general(p, v)
    assert abs(m.objective(red, v) - bf.objective_general(p, xs, us)) <= 1e-11


def check_general_rows(m):
    p = tg.case(*tg.CASES[1])
    red = m.reduce_problem(p)
    v = np.random.default_rng(5).normal(size=p.n)
    xs, us = bf.simulate_general(p, v)
    vals = bf.constraint_values(p, xs, us)
    got = red.J @ v - red.d
    for g, want in vals.items():
        np.testing.assert_allclose(got[red.groups == g], want[red.index[red.groups == g]],
                                   rtol=1e-11, atol=1e-12)


def check_general_active_set(m):
    for args in tg.TIGHT[:3]:
        p = tg.tight_case(*args)
        u_ex, f_ex = bf.sparse_active_set(p)
        r = m.solve(p, max_iter=60)
        assert r.status == 0
        assert np.max(np.abs(r.u - u_ex)) <= 1e-5


CHECKS = [check_simulation, check_objective, check_full_space, check_ftb, check_riccati,
          check_active_set, check_tight_converges, check_linear_residual_decay,
          check_barrier_rule, check_scalar_mu_sequence, check_shift, check_warm_start_point,
          check_closed_loop_lqr, check_general_simulation, check_general_objective,
          check_general_rows, check_general_active_set]


def run_checks(m):
    failed = []
    for chk in CHECKS:
        try:
            chk(m)
        except Exception:
            failed.append(chk.__name__)
    return failed


def test_unmutated_oracle_passes_all_checks():
    assert run_checks(load_variant(None)) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    with np.errstate(all="ignore"):
        failed = run_checks(load_variant(name))
    assert failed, f"mutation {name} escaped every pin"
