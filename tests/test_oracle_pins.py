"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a forward simulation, a closed form, an
exhaustive search, a different formulation of the same Newton step, or a size stated in the
paper.  None of these calls the GPU.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import condensed_ipm as ipm
from paper_2209_13049_amd import workloads as W
import brute_force as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_stable(ns, nu, N, seed, bound_x=0.5, bound_u=1.0, x0_scale=0.4, diagQ=False):
    rng = np.random.default_rng([99, seed])
    A = rng.normal(size=(ns, ns))
    A *= 0.9 / max(1e-12, np.max(np.abs(np.linalg.eigvals(A))))
    B = rng.normal(size=(ns, nu))
    M = rng.normal(size=(ns, ns))
    Q = np.diag(rng.uniform(0.5, 2.0, ns)) if diagQ else M @ M.T / ns + 0.5 * np.eye(ns)
    Mr = rng.normal(size=(nu, nu))
    R = Mr @ Mr.T / nu + 0.2 * np.eye(nu)
    Qf = 2.0 * Q
    x0 = rng.uniform(-x0_scale, x0_scale, ns)
    bx, bu = float(bound_x), float(bound_u)
    return W.LQProblem(A=A, B=B, Q=Q, R=R, Qf=Qf, xl=np.full(ns, -bx), xu=np.full(ns, bx),
                       ul=np.full(nu, -bu), uu=np.full(nu, bu), x0=x0, N=N)


# ---------------------------------------------------------------- reduction (Section 2)

@pytest.mark.parametrize("ns,nu,N,seed", [(1, 1, 1, 0), (3, 1, 4, 1), (4, 2, 5, 2), (6, 3, 3, 3),
                                          (5, 2, 1, 4)])
def test_reduction_reproduces_forward_simulation(ns, nu, N, seed):
    """c + Gamma v equals the simulated states x_1..x_N (eqn. (x_def) vs eqn. (dyn))."""
    p = random_stable(ns, nu, N, seed)
    red = oracle.reduce_problem(p)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        v = rng.normal(size=nu * N)
        x_sim = oracle.simulate(p, v)
        np.testing.assert_allclose(red.c + red.Gamma @ v, x_sim, rtol=1e-12, atol=1e-12)


def test_reduction_heat_small():
    p = W.heat1d_config("small")
    red = oracle.reduce_problem(p)
    v = np.random.default_rng(5).uniform(-1, 1, p.n)
    np.testing.assert_allclose(red.c + red.Gamma @ v, oracle.simulate(p, v), rtol=1e-12,
                               atol=1e-13)
    # Gamma is block lower-triangular: block (t, j) vanishes for j >= t
    ns, nu = p.ns, p.nu
    for t in range(1, p.N + 1):
        assert np.all(red.Gamma[(t - 1) * ns:t * ns, t * nu:] == 0)


@pytest.mark.parametrize("seed", range(4))
def test_dense_objective_equals_sparse_objective(seed):
    """1/2 v'Hv + h'v + h0 (eqn. (dense)) equals the simulated objective of eqn. (sparse)."""
    p = random_stable(3 + seed, 1 + seed % 3, 2 + seed, seed)
    red = oracle.reduce_problem(p)
    rng = np.random.default_rng(seed + 10)
    for _ in range(3):
        v = rng.normal(size=p.n)
        assert abs(oracle.objective(red, v) - oracle.sparse_objective(p, v)) <= \
            1e-12 * max(1.0, abs(oracle.sparse_objective(p, v)))


def test_hessian_symmetric_and_bounded_below():
    """H = Gamma'Qbar Gamma + Rbar is symmetric with lambda_min(H) >= lambda_min(R)."""
    for seed in range(3):
        p = random_stable(4, 2, 4, seed)
        red = oracle.reduce_problem(p)
        assert np.allclose(red.H, red.H.T, atol=0)
        lmin_R = np.linalg.eigvalsh(p.R).min()
        assert np.linalg.eigvalsh(red.H).min() >= lmin_R * (1 - 1e-12)


def test_sizes_stated_in_paper():
    """Sizes of Section 3 (condensed n_u T, augmented n_u T + 2(n_c+n_x+n_u)T) and the
    inequality count 2T(n_c+n_x+n_u) of eqn. (dense)."""
    cases = json.load(open(os.path.join(GOLDEN, "kkt_sizes.json")))["cases"]
    for c in cases:
        nx, nu, T = c["nx"], c["nu"], c["T"]
        assert nu * T == c["condensed"]
        assert nu * T + 2 * (c["nc"] + nx + nu) * T == c["augmented"]
        if nx * T * nu * T <= 5e6:
            p = W.heat1d(nx, nu, T) if nx >= nu else None
            red = oracle.reduce_problem(p)
            assert red.H.shape == (c["condensed"],) * 2
            assert red.J.shape[0] == c["inequalities"]
            # The size the paper states for the augmented system is n + m; the block system
            # of eqn. (aug_KKT) as printed has unknowns (p_v, p_s, p_lambda): n + 2m.
            assert red.H.shape[0] + red.J.shape[0] == c["augmented"]


def test_infinite_bounds_drop_rows():
    p = W.heat1d(6, 2, 3)
    p.xu[1] = np.inf
    p.ul[0] = -np.inf
    red = oracle.reduce_problem(p)
    full = 2 * (6 + 2) * 3
    assert red.J.shape[0] == full - 3 - 3
    assert np.all(np.isfinite(red.d))


# ------------------------------------------------------------ Newton step (Section 3)

def _interior_point(red, seed):
    rng = np.random.default_rng(seed)
    m = red.J.shape[0]
    v = rng.uniform(-0.3, 0.3, red.H.shape[0])
    s = rng.uniform(0.05, 1.5, m)
    lam = rng.uniform(0.01, 2.0, m)
    z = rng.uniform(0.01, 2.0, m)
    return v, s, lam, z, float(rng.uniform(1e-3, 0.1))


@pytest.mark.parametrize("ns,nu,N,seed", [(2, 1, 2, 0), (3, 1, 3, 1), (3, 2, 2, 2),
                                          (2, 2, 3, 3)])
def test_condensed_step_equals_full_space_newton(ns, nu, N, seed):
    """The condensed direction equals the Newton direction of the sparse problem (states as
    variables, dynamics as equality constraints, assembled from A, B, Q, R)."""
    p = random_stable(ns, nu, N, seed)
    p.xu[0] = np.inf          # one missing bound, so dropped rows are covered too
    red = oracle.reduce_problem(p)
    v, s, lam, z, mu = _interior_point(red, seed)
    step = oracle.condensed_step(red, v, s, lam, z, mu)
    pu, ps, plam, pz = bf.full_space_step(p, v, s, lam, z, mu)
    scale = 1.0 + np.max(np.abs(pu))
    np.testing.assert_allclose(step["pv"], pu, rtol=1e-9, atol=1e-10 * scale)
    np.testing.assert_allclose(step["ps"], ps, rtol=1e-9, atol=1e-10 * scale)
    np.testing.assert_allclose(step["plam"], plam, rtol=1e-9, atol=1e-9 * (1 + np.abs(plam).max()))
    np.testing.assert_allclose(step["pz"], pz, rtol=1e-9, atol=1e-9 * (1 + np.abs(pz).max()))


@pytest.mark.parametrize("seed", range(3))
def test_condensed_step_equals_augmented_system(seed):
    p = random_stable(3, 2, 3, seed)
    red = oracle.reduce_problem(p)
    v, s, lam, z, mu = _interior_point(red, seed)
    step = oracle.condensed_step(red, v, s, lam, z, mu)
    pv, ps, plam = bf.augmented_step(red.H, red.h, red.J, red.d, v, s, lam, mu, z)
    np.testing.assert_allclose(step["pv"], pv, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(step["ps"], ps, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(step["plam"], plam, rtol=1e-9, atol=1e-10)


def test_condensed_matrix_spd():
    """K = H + J'Sigma J with Sigma > 0 is SPD with lambda_min(K) >= lambda_min(R)."""
    p = W.heat1d_config("small")
    red = oracle.reduce_problem(p)
    rng = np.random.default_rng(1)
    lmin_R = np.linalg.eigvalsh(p.R).min()
    for scale in (1e-9, 1.0, 1e9):
        sigma = scale * rng.uniform(0.1, 10, red.J.shape[0])
        K = oracle.condensed_matrix(red, sigma)
        assert np.linalg.eigvalsh(K).min() >= lmin_R * (1 - 1e-12) * 0.999
        np.linalg.cholesky(K)


def test_fraction_to_boundary_closed_form():
    s = np.array([1.0, 2.0, 0.5, 3.0])
    p = np.array([-2.0, 1.0, -0.1, -0.5])
    # candidates: 0.99*1/2 = 0.495, 0.99*0.5/0.1 = 4.95, 0.99*3/0.5 = 5.94 -> 0.495
    assert oracle.fraction_to_boundary(s, p, 0.99) == pytest.approx(0.495, rel=1e-15)
    assert oracle.fraction_to_boundary(s, np.abs(p), 0.99) == 1.0


# --------------------------------------------------------- converged result (Alg. 1)

@pytest.mark.parametrize("ns,nu,N,seed", [(3, 1, 4, 0), (4, 2, 6, 1), (6, 3, 5, 2)])
def test_unconstrained_matches_riccati(ns, nu, N, seed):
    """With bounds that never bind (+-1e3), the IPM solution is the LQR solution."""
    p = random_stable(ns, nu, N, seed, bound_x=1e3, bound_u=1e3)
    r = oracle.solve(p)
    assert r.status == oracle.STATUS_CONVERGED
    u_ric, f_ric = bf.riccati(p)
    assert np.max(np.abs(r.v - u_ric)) <= 1e-7 * max(1.0, np.max(np.abs(u_ric)))
    assert abs(r.obj - f_ric) <= 1e-9 * max(1.0, abs(f_ric))


def test_unconstrained_heat_small_matches_riccati():
    p = W.heat1d_config("small")
    p.xu[:] = 1e3
    p.xl[:] = -1e3
    p.uu[:] = 1e3
    p.ul[:] = -1e3
    r = oracle.solve(p)
    u_ric, f_ric = bf.riccati(p)
    assert r.status == 0
    assert np.max(np.abs(r.v - u_ric)) <= 1e-7 * max(1.0, np.max(np.abs(u_ric)))
    assert abs(r.obj - f_ric) <= 1e-9 * abs(f_ric)


def test_scalar_golden_cases():
    """Hand-worked one-step problems (golden/scalar_lq.json) and the closed-form clamp."""
    cases = json.load(open(os.path.join(GOLDEN, "scalar_lq.json")))["cases"]
    for c in cases:
        u_cf, f_cf = bf.scalar_clamp(c["a"], c["b"], c["q"], c["qf"], c["r"], c["x0"],
                                     c["xl"], c["xu"], c["ul"], c["uu"])
        assert u_cf == pytest.approx(c["u"], abs=1e-15)
        assert f_cf == pytest.approx(c["f"], rel=1e-14)
        p = W.LQProblem(A=np.array([[c["a"]]]), B=np.array([[c["b"]]]),
                        Q=np.array([[c["q"]]]), R=np.array([[c["r"]]]),
                        Qf=np.array([[c["qf"]]]), xl=np.array([c["xl"]]),
                        xu=np.array([c["xu"]]), ul=np.array([c["ul"]]),
                        uu=np.array([c["uu"]]), x0=np.array([c["x0"]]), N=1)
        r = oracle.solve(p)
        assert r.status == 0
        assert r.v[0] == pytest.approx(c["u"], abs=1e-7)
        assert r.x[0] == pytest.approx(c["x1"], abs=1e-7)
        assert r.obj == pytest.approx(c["f"], rel=1e-7)


@pytest.mark.parametrize("seed", range(8))
def test_scalar_random_clamp(seed):
    rng = np.random.default_rng([7, seed])
    a, b = rng.uniform(-1.2, 1.2), rng.uniform(0.2, 2.0)
    q, qf, r = rng.uniform(0.1, 2), rng.uniform(0.1, 3), rng.uniform(0.05, 1)
    x0 = rng.uniform(-1, 1)
    ul, uu = -rng.uniform(0.05, 1), rng.uniform(0.05, 1)
    xl, xu = -rng.uniform(0.1, 2), rng.uniform(0.1, 2)
    x0 = float(np.clip(x0, xl + 0.05, xu - 0.05))
    lo, hi = max(ul, (xl - a * x0) / b), min(uu, (xu - a * x0) / b)
    if lo >= hi - 1e-3:
        pytest.skip("empty feasible interval for this draw")
    u_cf, f_cf = bf.scalar_clamp(a, b, q, qf, r, x0, xl, xu, ul, uu)
    p = W.LQProblem(A=np.array([[a]]), B=np.array([[b]]), Q=np.array([[q]]),
                    R=np.array([[r]]), Qf=np.array([[qf]]), xl=np.array([xl]),
                    xu=np.array([xu]), ul=np.array([ul]), uu=np.array([uu]),
                    x0=np.array([x0]), N=1)
    res = oracle.solve(p)
    assert res.status == 0
    assert res.v[0] == pytest.approx(u_cf, abs=1e-7)
    assert res.obj == pytest.approx(f_cf, rel=1e-7, abs=1e-9)


def _pairs(red, ns, nu, N):
    """(upper row, lower row) index pairs per bounded quantity of the oracle's J."""
    rows = {}
    for k, (g, i) in enumerate(zip(red.groups, red.index)):
        key = ("x" if g < 2 else "u", int(i))
        rows.setdefault(key, [None, None])[0 if g in (0, 2) else 1] = k
    return [tuple(v) for v in rows.values()]


def _binding_case(seed, kind):
    """Tiny problems (ns=2, nu=1, N=3) built so that bounds bind at the optimum:
    'u': control bounds at 60% of the unconstrained (Riccati) control magnitude;
    'x': a positive first state with a lower bound at half its start value, which the
    controller, pulling the state to zero, must respect."""
    p = random_stable(2, 1, 3, seed, bound_x=10.0, bound_u=10.0, x0_scale=1.0)
    if kind == "u":
        u_ric, _ = bf.riccati(p)
        p.uu[:] = 0.6 * np.max(np.abs(u_ric))
        p.ul[:] = -p.uu
    else:
        p.x0[0] = abs(p.x0[0]) + 0.2
        p.xl[0] = 0.5 * p.x0[0]
    return p


@pytest.mark.parametrize("seed,kind", [(40, "u"), (43, "u"), (45, "u"), (47, "u"),
                                       (40, "x"), (43, "x"), (46, "x")])
def test_active_set_enumeration(seed, kind):
    """Binding bounds: the IPM solution equals the exhaustive active-set solution, and its
    objective exceeds the exact one by no more than the final duality gap s'z."""
    p = _binding_case(seed, kind)
    red = oracle.reduce_problem(p)
    r = oracle.solve(p)
    assert r.status == 0
    v_ex, lam_ex = bf.active_set(red.H, red.h, red.J, red.d, _pairs(red, 2, 1, 3))
    f_ex = oracle.objective(red, v_ex)
    active = np.where(lam_ex > 1e-9)[0]
    assert len(active) >= 1, "the case should have a binding bound"
    assert set(red.groups[active]) <= ({2, 3} if kind == "u" else {0, 1})
    assert r.obj >= f_ex - 1e-12 and r.obj - f_ex <= r.gap + 1e-12
    assert np.max(np.abs(r.v - v_ex)) <= 1e-4


def test_iteration_invariants_tight():
    """Along the iteration: s > 0, z > 0; r3 shrinks by exactly (1 - alpha) (linear
    constraints); the safeguard keeps s z / mu in [1/kappa, kappa]; K is SPD."""
    p = W.heat1d(40, 4, 8, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    red = oracle.reduce_problem(p)
    lmin_R = np.linalg.eigvalsh(p.R).min()
    log = []

    def cb(st):
        log.append(st)
    r = oracle.solve(p, red=red, callback=cb)
    assert r.status == 0
    assert len(log) >= 5
    for a, b in zip(log[:-1], log[1:]):
        assert np.all(b["s"] > 0) and np.all(b["z"] > 0)
        np.testing.assert_allclose(b["r3"], (1 - a["alpha"]) * a["r3"], atol=1e-12)
        ratio = b["s"] * b["z"] / a["mu"] if b["mu"] == a["mu"] else None
        if ratio is not None:
            assert ratio.min() >= 1 / ipm.KAPPA_SIGMA * (1 - 1e-12)
            assert ratio.max() <= ipm.KAPPA_SIGMA * (1 + 1e-12)
    for st in log[::3]:
        assert np.linalg.eigvalsh(st["K"]).min() >= lmin_R * 0.999


def test_infeasible_start_reduces_r3_linearly():
    """A start with d - Jv < 1e-2 on some rows gives r3 != 0, which then decays by (1 - alpha)."""
    p = W.heat1d(20, 2, 5, seed=(5, 0), xu=0.05, x0_range=(0.045, 0.05))
    red = oracle.reduce_problem(p)
    log = []
    r = oracle.solve(p, red=red, callback=log.append)
    assert np.max(np.abs(log[0]["r3"])) > 1e-4
    for a, b in zip(log[:-1], log[1:]):
        np.testing.assert_allclose(b["r3"], (1 - a["alpha"]) * a["r3"], atol=1e-12)
        # r1 = Hv + h + J'lambda is affine in (v, lambda), which share the step length
        np.testing.assert_allclose(b["r1"], (1 - a["alpha"]) * a["r1"], atol=1e-10)
    assert r.status == 0 and r.primal_res <= 1e-8


@pytest.mark.slow
def test_config_1d_no_bound_active_matches_riccati():
    """The 1000-state workload: no bound binds at its optimum, so the LQR solution is the
    answer up to the barrier term (objective within the final duality gap)."""
    p = W.heat1d_config("1d")
    r = oracle.solve(p)
    u_ric, f_ric = bf.riccati(p)
    assert r.status == 0
    assert np.max(np.abs(u_ric)) < 1.0 and np.max(np.abs(oracle.simulate(p, u_ric))) < 0.5
    assert r.obj >= f_ric - 1e-9 * abs(f_ric)
    assert r.obj - f_ric <= r.gap


def test_heat3d_generator_table1():
    """The 3-D cube of Section 5 with Table 1's constants: r = k dt / (rho cp dw^2); a uniform
    temperature with every face at that temperature is a steady state (A 1 + B 1 = 1); each face
    touches m^2 interior nodes; the step is symmetric and stable."""
    m = 4
    A, B = W.heat3d_dynamics(m)
    r = 400.0 * 0.1 / (8960.0 * 386.0 * 0.02 ** 2)
    ns = m ** 3
    assert np.allclose(A, A.T, rtol=0, atol=0)
    assert np.max(np.abs(A @ np.ones(ns) + B @ np.ones(6) - 1.0)) < 1e-14
    assert np.allclose(B.sum(axis=0), r * m * m, rtol=1e-14)
    centre = (1 * m + 1) * m + 1  # node (1, 1, 1): all 6 neighbours interior
    assert np.all(B[centre] == 0.0) and A[centre, centre] == pytest.approx(1.0 - 6.0 * r)
    corner = 0  # node (0, 0, 0): faces x = 0, y = 0, z = 0
    assert np.count_nonzero(B[corner]) == 3 and B[corner, 0] == B[corner, 2] == B[corner, 4] == r
    assert np.max(np.abs(np.linalg.eigvals(A))) < 1.0
    p = W.heat3d(m, 5)
    assert np.all(p.x0 == 300.0 - 400.0) and np.all(p.xl == -200.0) and np.all(p.xu == 150.0)
    assert np.all(p.ul == -100.0) and np.all(p.uu == 100.0)
    assert p.Q[0, 0] == pytest.approx(10 * 0.02 ** 2) and p.R[0, 0] == pytest.approx(0.1 * 0.02 ** 2)


def test_heat3d_solution_has_the_cube_symmetry():
    """Uniform initial state, set point and bounds: the optimum is invariant under the cube's
    symmetries, so all six faces get the same input at every step (a misplaced face column of
    B breaks this); heating from 300 K toward 400 K saturates the inputs at the start."""
    p = W.heat3d(3, 6)
    res = ipm.solve(p)
    assert res.status == 0
    u = np.asarray(res.v).reshape(p.N, 6)
    assert np.max(u.max(axis=1) - u.min(axis=1)) < 1e-6
    assert np.all(u[0] == pytest.approx(100.0, abs=1e-6))
