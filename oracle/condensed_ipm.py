"""Plain FP64 CPU oracle of the condensed-space interior-point method for LQ-MPC.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this package; the HIP library and
its Python binding never do, and this package imports nothing from them.

It follows Cole, Shin, Pacaud, Zavala and Anitescu, "Exploiting GPU/SIMD architectures for
solving linear-quadratic MPC problems" (arXiv 2209.13049):

* ``reduce_problem``  -- Section 2, eqns. (K_constraint), (x_def) and (dense): eliminate the
  states, giving min 1/2 v'Hv + h'v + h0  s.t.  Jv <= d (``reduce_general`` for problems
  with a cross weight S, rows g^l <= E x + F u <= g^u, a disturbance w or a feedback K).
* ``condensed_step``  -- Section 3, eqns. (aug_KKT) and (cond_KKT) and the recovery
  formulas that follow them: one Newton step through the condensed matrix H + J'Sigma J,
  factored by dense Cholesky.
* ``barrier_update``  -- the barrier-parameter rule that Algorithm 1 leaves open (R8).
* ``solve``           -- Algorithm 1 (condensed-space IPM), with the readings listed below.

Everything is written from the definitions, in float64, with numpy/scipy primitives
(matrix products, Cholesky) as steps and no blocking or reordering.

Readings where the paper is silent or ambiguous (each one is also exercised by a test):

R1  Objective carries a 1/2 on every quadratic term (eqn. (dense) and the PDE objective
    have it; eqn. (sparse) does not; the minimiser is the same).
R2  Q_f defaults to Q.
R3  State-bound rows at t = 0 are constants and are dropped; bounds apply for t = 1..N.
    Rows whose bound is infinite are dropped.
R4  Stabilising feedback K = 0 (v = u) unless the problem gives one (``reduce_general``).
R5  The right-hand side of eqn. (cond_KKT) is -r1 + J'r2 - J'Sigma r3 (the printed "J r2"
    is read as J'r2, which the block elimination of eqn. (aug_KKT) gives).
R6  Sigma in the p^z formula of Algorithm 1 is Sigma_s = S^-1 Z.
R7  Start: mu = 0.1, v = 0, s = max(d - Jv, 1e-2), lambda = z = mu / s.
R8  Barrier parameter: monotone (Fiacco-McCormick) rule of Waechter and Biegler's IPOPT
    paper, with kappa_eps = 10, kappa_mu = 0.2, theta_mu = 1.5, mu_min = tol / 10.
R9  "Line search" = fraction-to-the-boundary step lengths alpha (for v, s, lambda) and
    alpha_z (for z) with tau = max(0.99, 1 - mu); no merit backtracking (the problem is a
    convex QP with linear constraints).
R10 After each update z is safeguarded into [mu / (kappa_S s), kappa_S mu / s],
    kappa_S = 1e10.
R11 Termination: E_0 = max(|r1|, |r3|, |lambda - z|, |s z|) <= tol (unscaled inf-norms),
    checked at the top of every iteration; iteration limit 200.
R14 Receding horizon (Section 1: the controller solves the problem from each measured state
    and applies the first input): a solve may start from given controls v0 instead of 0,
    with s, lambda and z as in R7 at that v0 and the barrier parameter starting at
    WARM_MU_INIT = 1e-3; the warm start of the next step is the previous step's controls
    shifted one stage earlier, the last stage repeated (``shift_controls``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

KAPPA_EPS = 10.0
KAPPA_MU = 0.2
THETA_MU = 1.5
KAPPA_SIGMA = 1e10
TAU_MIN = 0.99
MU_INIT = 0.1
WARM_MU_INIT = 1e-3
S_INIT_MIN = 1e-2
ALPHA_MIN = 1e-14

STATUS_CONVERGED = 0
STATUS_MAX_ITER = 1
STATUS_SMALL_STEP = 2


@dataclass
class Reduced:
    """The dense QP of eqn. (dense) plus the pieces of eqn. (x_def) it was built from."""

    Gamma: np.ndarray      # (ns N) x (nu N): block (t, j) = A^(t-1-j) B for j < t, t = 1..N
    c: np.ndarray          # (ns N): free response A^t x0, t = 1..N
    Rbar: np.ndarray       # block diag(R, ..., R) over t = 0..N-1
    H: np.ndarray
    h: np.ndarray
    h0: float
    J: np.ndarray          # inequality rows that are kept (finite bounds)
    d: np.ndarray
    groups: np.ndarray     # 0: x <= xu, 1: -x <= -xl, 2: u <= uu, 3: -u <= -ul,
                           # 4: Ex + Fu <= gu, 5: -(Ex + Fu) <= -gl (kept rows)
    index: np.ndarray      # row index inside its group (kept rows)
    u0: np.ndarray | None = None   # inputs u = u0 + Uv (None: u = v)
    Uv: np.ndarray | None = None


def inputs(red: Reduced, v: np.ndarray) -> np.ndarray:
    """The inputs u_t = K x_t + v_t of eqn. (K_constraint), stacked (u = v when K = 0)."""
    return v.copy() if red.Uv is None else red.u0 + red.Uv @ v


def powers_times(A: np.ndarray, X: np.ndarray, N: int):
    """[X, A X, A^2 X, ..., A^N X] by repeated multiplication (A^k X, k = 0..N)."""
    out = [np.array(X, dtype=np.float64)]
    for _ in range(N):
        out.append(A @ out[-1])
    return out


def reduce_problem(prob) -> Reduced:
    """State elimination of Section 2 (eqn. (x_def)) with K = 0 and w = 0 (problems with
    more data go to ``reduce_general``).

    x = bA x0 + bB v, where bA stacks A^t and bB is block lower-triangular with block
    (t, j) = A^(t-1-j) B.  Rows of x_0 (t = 0) are constants and are not kept (reading R3).
    Substituting into the objective (reading R1: 1/2 convention) gives
        H = bB' Qbar bB + Rbar,  h = bB' Qbar c,  h0 = 1/2 x0'Q x0 + 1/2 c'Qbar c,
    with c = (A^t x0)_{t=1..N} and Qbar = blockdiag(Q, ..., Q, Q_f), and the inequalities
    J v <= d with J = [Gamma; -Gamma; I; -I],  d = [xu - c; c - xl; uu; -ul].
    Qbar is block diagonal, so it is applied block by block instead of being formed.
    """
    if getattr(prob, "general", False):
        return reduce_general(prob)
    A, B, Q, R, Qf = prob.A, prob.B, prob.Q, prob.R, prob.Qf
    ns, nu, N = A.shape[0], B.shape[1], int(prob.N)
    G = powers_times(A, B, N - 1)                      # G[k] = A^k B
    xs = powers_times(A, prob.x0, N)                   # xs[t] = A^t x0
    Gamma = np.zeros((ns * N, nu * N))
    for t in range(1, N + 1):
        for j in range(t):
            Gamma[(t - 1) * ns:t * ns, j * nu:(j + 1) * nu] = G[t - 1 - j]
    c = np.concatenate(xs[1:])

    def qbar_times(X):
        """Qbar X for X with ns N rows."""
        out = np.empty_like(X)
        for t in range(1, N + 1):
            W = Qf if t == N else Q
            out[(t - 1) * ns:t * ns] = W @ X[(t - 1) * ns:t * ns]
        return out

    Rbar = np.kron(np.eye(N), R)
    H = Gamma.T @ qbar_times(Gamma) + Rbar
    H = 0.5 * (H + H.T)
    h = Gamma.T @ qbar_times(c)
    h0 = 0.5 * prob.x0 @ Q @ prob.x0 + 0.5 * c @ qbar_times(c)
    I = np.eye(nu * N)
    xu = np.tile(prob.xu, N)
    xl = np.tile(prob.xl, N)
    uu = np.tile(prob.uu, N)
    ul = np.tile(prob.ul, N)
    J_all = np.vstack([Gamma, -Gamma, I, -I])
    d_all = np.concatenate([xu - c, c - xl, uu, -ul])
    g_all = np.concatenate([np.full(ns * N, 0), np.full(ns * N, 1), np.full(nu * N, 2),
                            np.full(nu * N, 3)])
    i_all = np.concatenate([np.arange(ns * N), np.arange(ns * N), np.arange(nu * N),
                            np.arange(nu * N)])
    keep = np.isfinite(d_all)
    return Reduced(Gamma=Gamma, c=c, Rbar=Rbar, H=H, h=h, h0=float(h0),
                   J=J_all[keep], d=d_all[keep], groups=g_all[keep], index=i_all[keep])


def reduce_general(prob) -> Reduced:
    """State elimination of Section 2 with every kind of data of eqn. (sparse).

    Feedback (eqn. (K_constraint)): u_t = K x_t + v_t, so x_{t+1} = A_K x_t + B v_t + w_t with
    A_K = A + B K, and eqn. (x_def) is x_t = c_t + Gamma_t v: c_0 = x0, c_{t+1} = A_K c_t + w_t;
    Gamma_0 = 0, Gamma_{t+1} = A_K Gamma_t + B [block t of v] (block j of Gamma_t is
    A_K^(t-1-j) B).  The inputs are u_t = K c_t + (K Gamma_t + [block t]) v.
    Objective of eqn. (sparse), 1/2 convention: with z the stack of (x_t, u_t), t = 0..N-1,
    and x_N, an affine function z = z0 + Z v, the objective is 1/2 z' W z with
    W = blockdiag([[Q, S], [S', R]], ..., Q_f); hence H = Z' W Z, h = Z' W z0 and
    h0 = 1/2 z0' W z0.  Inequalities: x_t in [xl, xu] for t = 1..N (reading R3), u_t in
    [ul, uu] and E x_t + F u_t in [gl, gu] for t = 0..N-1, each an affine row of v.
    """
    A, B, Q, R, Qf = prob.A, prob.B, prob.Q, prob.R, prob.Qf
    ns, nu, N = A.shape[0], B.shape[1], int(prob.N)
    n = nu * N
    K = np.zeros((nu, ns)) if prob.Kfb is None else np.asarray(prob.Kfb, dtype=np.float64)
    S = np.zeros((ns, nu)) if prob.S is None else np.asarray(prob.S, dtype=np.float64)
    w = np.zeros((N, ns)) if prob.w is None else np.asarray(prob.w, dtype=np.float64)
    AK = A + B @ K
    # x_t = X0[t] + XV[t] v, u_t = U0[t] + UV[t] v
    X0 = [np.array(prob.x0, dtype=np.float64)]
    XV = [np.zeros((ns, n))]
    U0, UV = [], []
    for t in range(N):
        sel = np.zeros((nu, n))
        sel[:, t * nu:(t + 1) * nu] = np.eye(nu)
        U0.append(K @ X0[t])
        UV.append(K @ XV[t] + sel)
        X0.append(AK @ X0[t] + w[t])
        XV.append(AK @ XV[t] + B @ sel)
    # objective: z = (x_0, u_0, x_1, u_1, ..., x_{N-1}, u_{N-1}, x_N)
    z0 = np.concatenate([np.concatenate([X0[t], U0[t]]) for t in range(N)] + [X0[N]])
    Z = np.vstack([np.vstack([XV[t], UV[t]]) for t in range(N)] + [XV[N]])
    Wst = np.block([[Q, S], [S.T, R]])
    Wbar = sla.block_diag(*([Wst] * N + [Qf]))
    H = Z.T @ Wbar @ Z
    H = 0.5 * (H + H.T)
    h = Z.T @ Wbar @ z0
    h0 = 0.5 * z0 @ Wbar @ z0
    Gamma = np.vstack(XV[1:])
    c = np.concatenate(X0[1:])
    Uv = np.vstack(UV)
    u0 = np.concatenate(U0)
    blocks = [(Gamma, np.tile(prob.xu, N) - c, 0), (-Gamma, c - np.tile(prob.xl, N), 1),
              (Uv, np.tile(prob.uu, N) - u0, 2), (-Uv, u0 - np.tile(prob.ul, N), 3)]
    if prob.E is not None:
        E, F = np.asarray(prob.E, dtype=np.float64), np.asarray(prob.F, dtype=np.float64)
        Cv = np.vstack([E @ XV[t] + F @ UV[t] for t in range(N)])
        c0 = np.concatenate([E @ X0[t] + F @ U0[t] for t in range(N)])
        blocks += [(Cv, np.tile(prob.gu, N) - c0, 4), (-Cv, c0 - np.tile(prob.gl, N), 5)]
    J_all = np.vstack([b[0] for b in blocks])
    d_all = np.concatenate([b[1] for b in blocks])
    g_all = np.concatenate([np.full(b[0].shape[0], b[2]) for b in blocks])
    i_all = np.concatenate([np.arange(b[0].shape[0]) for b in blocks])
    keep = np.isfinite(d_all)
    return Reduced(Gamma=Gamma, c=c, Rbar=np.kron(np.eye(N), R), H=H, h=h, h0=float(h0),
                   J=J_all[keep], d=d_all[keep], groups=g_all[keep], index=i_all[keep],
                   u0=u0, Uv=Uv)


def objective(red: Reduced, v: np.ndarray) -> float:
    """1/2 v'Hv + h'v + h0 (eqn. (dense))."""
    return float(0.5 * v @ red.H @ v + red.h @ v + red.h0)


def residuals(red: Reduced, v, s, lam, mu):
    """r1, r2, r3 as defined under eqn. (aug_KKT)."""
    r1 = red.H @ v + red.h + red.J.T @ lam
    r2 = lam - mu / s
    r3 = red.J @ v - red.d + s
    return r1, r2, r3


def condensed_matrix(red: Reduced, sigma: np.ndarray) -> np.ndarray:
    """H + J' Sigma_s J (left-hand side of eqn. (cond_KKT))."""
    return red.H + red.J.T @ (sigma[:, None] * red.J)


def condensed_step(red: Reduced, v, s, lam, z, mu):
    """One Newton direction through the condensed system (Section 3).

    Sigma_s = S^-1 Z; (H + J'Sigma J) p_v = -r1 + J'r2 - J'Sigma r3 (reading R5), solved by
    Cholesky; p_s = -r3 - J p_v; p_lambda = -r2 + Sigma r3 + Sigma J p_v;
    p_z = mu S^-1 1 - z - Sigma p_s (reading R6).
    """
    sigma = z / s
    r1, r2, r3 = residuals(red, v, s, lam, mu)
    K = condensed_matrix(red, sigma)
    rhs = -r1 + red.J.T @ r2 - red.J.T @ (sigma * r3)
    factor = sla.cho_factor(K, lower=True)
    pv = sla.cho_solve(factor, rhs)
    Jpv = red.J @ pv
    ps = -r3 - Jpv
    plam = -r2 + sigma * r3 + sigma * Jpv
    pz = mu / s - z - sigma * ps
    return dict(pv=pv, ps=ps, plam=plam, pz=pz, sigma=sigma, K=K, rhs=rhs, r1=r1, r2=r2, r3=r3)


def fraction_to_boundary(x: np.ndarray, p: np.ndarray, tau: float) -> float:
    """Largest alpha in (0, 1] with x + alpha p >= (1 - tau) x (reading R9)."""
    neg = p < 0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-tau * x[neg] / p[neg])))


def optimality_error(r1, r3, lam, z, s, mu):
    """E_mu = max(|r1|, |r3|, |lambda - z|, |s z - mu|) in the inf-norm (readings R8, R11).

    r1 is the stationarity residual and r3 the primal residual defined under eqn. (aug_KKT);
    lambda - z is the mismatch of the two multipliers of a row (stationarity in s) and
    s z - mu the perturbed complementarity.  Returns (E_mu, [the four norms]).
    """
    parts = [np.max(np.abs(r1), initial=0.0), np.max(np.abs(r3), initial=0.0),
             np.max(np.abs(lam - z), initial=0.0), np.max(np.abs(s * z - mu), initial=0.0)]
    return float(max(parts)), parts


def kkt_error(red: Reduced, v, s, lam, z, mu):
    """E_mu at the iterate (v, s, lambda, z) of the dense QP (see optimality_error)."""
    r1 = red.H @ v + red.h + red.J.T @ lam
    r3 = red.J @ v - red.d + s
    return optimality_error(r1, r3, lam, z, s, mu)


def barrier_update(mu, r1, r3, lam, z, s, mu_min):
    """Monotone (Fiacco-McCormick) barrier rule of reading R8, applied at the top of an
    iteration after the stop test.

    While mu > mu_min and the barrier problem of the current mu is solved to
    E_mu <= KAPPA_EPS mu, move to mu <- max(mu_min, min(KAPPA_MU mu, mu^THETA_MU)); the
    residuals r1, r3 do not depend on mu, only the complementarity term of E_mu does.
    Returns (mu, tau) with the fraction-to-boundary parameter tau = max(TAU_MIN, 1 - mu)
    of the new mu (reading R9).
    """
    while mu > mu_min:
        emu, _ = optimality_error(r1, r3, lam, z, s, mu)
        if emu > KAPPA_EPS * mu:
            break
        mu = max(mu_min, min(KAPPA_MU * mu, mu ** THETA_MU))
    return mu, max(TAU_MIN, 1.0 - mu)


@dataclass
class Result:
    status: int
    iters: int
    v: np.ndarray
    s: np.ndarray
    lam: np.ndarray
    z: np.ndarray
    mu: float
    obj: float
    primal_res: float
    dual_res: float
    compl_res: float
    gap: float
    x: np.ndarray
    history: list = field(default_factory=list)
    u: np.ndarray | None = None   # the inputs u = K x + v (= v when K = 0)


def initial_point(red: Reduced, mu0: float = MU_INIT, v0=None):
    """Reading R7 (v0 = None: v = 0), or reading R14 from the controls v0."""
    n = red.H.shape[0]
    v = np.zeros(n) if v0 is None else np.array(v0, dtype=np.float64)
    s = np.maximum(red.d - red.J @ v, S_INIT_MIN)
    lam = mu0 / s
    z = lam.copy()
    return v, s, lam, z


def solve(prob, tol: float = 1e-8, max_iter: int = 200, red: Reduced | None = None,
          callback=None, record: bool = False, v0=None, mu0: float | None = None) -> Result:
    """Algorithm 1 (condensed-space interior-point method) with readings R7-R11; v0 starts
    from given controls (reading R14, barrier parameter mu0, default WARM_MU_INIT)."""
    if red is None:
        red = reduce_problem(prob)
    mu = (MU_INIT if v0 is None else WARM_MU_INIT) if mu0 is None else mu0
    mu_min = tol / 10.0
    v, s, lam, z = initial_point(red, mu, v0)
    history = []
    status, k = STATUS_MAX_ITER, 0
    for k in range(max_iter + 1):
        e0, parts0 = kkt_error(red, v, s, lam, z, 0.0)
        if e0 <= tol:
            status = STATUS_CONVERGED
            break
        if k == max_iter:
            status = STATUS_MAX_ITER
            break
        # barrier update (reading R8)
        mu, tau = barrier_update(mu, red.H @ v + red.h + red.J.T @ lam,
                                 red.J @ v - red.d + s, lam, z, s, mu_min)
        step = condensed_step(red, v, s, lam, z, mu)
        alpha = fraction_to_boundary(s, step["ps"], tau)
        alpha_z = fraction_to_boundary(z, step["pz"], tau)
        if callback is not None:
            callback(dict(k=k, v=v, s=s, lam=lam, z=z, mu=mu, tau=tau, alpha=alpha,
                          alpha_z=alpha_z, **step))
        if record:
            history.append(dict(k=k, mu=mu, alpha=alpha, alpha_z=alpha_z, err=e0))
        if alpha < ALPHA_MIN:
            status = STATUS_SMALL_STEP
            break
        v = v + alpha * step["pv"]
        s = s + alpha * step["ps"]
        lam = lam + alpha * step["plam"]
        z = z + alpha_z * step["pz"]
        # safeguard (reading R10)
        z = np.minimum(np.maximum(z, mu / (KAPPA_SIGMA * s)), KAPPA_SIGMA * mu / s)
    r1 = red.H @ v + red.h + red.J.T @ lam
    r3 = red.J @ v - red.d + s
    x = red.c + red.Gamma @ v
    return Result(status=status, iters=k, v=v, s=s, lam=lam, z=z, mu=mu,
                  obj=objective(red, v), primal_res=float(np.max(np.abs(r3), initial=0.0)),
                  dual_res=float(np.max(np.abs(r1), initial=0.0)),
                  compl_res=float(np.max(np.abs(s * z), initial=0.0)), gap=float(s @ z),
                  x=x, history=history, u=inputs(red, v))


def simulate(prob, u: np.ndarray) -> np.ndarray:
    """Forward simulation x_{t+1} = A x_t + B u_t + w_t, t = 0..N-1 (eqn. (dyn); w = 0 when
    the problem has none), for the inputs u.

    Returns the states x_1..x_N stacked (length ns N).
    """
    ns, nu, N = prob.A.shape[0], prob.B.shape[1], int(prob.N)
    w = getattr(prob, "w", None)
    x = prob.x0.copy()
    out = []
    for t in range(N):
        x = prob.A @ x + prob.B @ u[t * nu:(t + 1) * nu]
        if w is not None:
            x = x + w[t]
        out.append(x)
    return np.concatenate(out)


def sparse_objective(prob, u: np.ndarray) -> float:
    """Objective of eqn. (sparse) with the 1/2 convention (reading R1), by simulation, for
    the inputs u (with the cross weight S where the problem has one)."""
    ns, nu, N = prob.A.shape[0], prob.B.shape[1], int(prob.N)
    S = getattr(prob, "S", None)
    xs = np.concatenate([prob.x0, simulate(prob, u)])
    f = 0.0
    for t in range(N):
        xt, ut = xs[t * ns:(t + 1) * ns], u[t * nu:(t + 1) * nu]
        f += 0.5 * xt @ prob.Q @ xt + 0.5 * ut @ prob.R @ ut
        if S is not None:
            f += xt @ S @ ut
    xN = xs[N * ns:]
    f += 0.5 * xN @ prob.Qf @ xN
    return float(f)


def shift_controls(v: np.ndarray, nu: int, N: int) -> np.ndarray:
    """Warm start of the next receding-horizon step (reading R14): stage t of the result is
    stage t + 1 of v (t = 0..N-2), and the last stage repeats stage N-1 of v."""
    v = np.asarray(v, dtype=np.float64)
    return np.concatenate([v[nu:nu * N], v[nu * (N - 1):nu * N]])


def closed_loop(prob, steps: int, warm: bool = True, tol: float = 1e-8):
    """Receding-horizon control of the model itself (Section 1): from x0, solve, apply the
    first input u_0, step the dynamics x+ = A x + B u_0, and solve again from x+; with
    warm, each solve after the first starts from the previous controls shifted
    (reading R14).  Returns the states x_0..x_steps, the applied inputs and the results."""
    from dataclasses import replace
    assert not getattr(prob, "general", False), "closed_loop takes problems without S, E, F, w, K"
    nu, N = prob.B.shape[1], int(prob.N)
    x = np.array(prob.x0, dtype=np.float64)
    xs, us, results = [x.copy()], [], []
    v_prev = None
    for _ in range(steps):
        p = replace(prob, x0=x.copy())
        v0 = shift_controls(v_prev, nu, N) if (warm and v_prev is not None) else None
        r = solve(p, tol=tol, v0=v0)
        results.append(r)
        u0 = r.v[:nu].copy()
        us.append(u0)
        x = prob.A @ x + prob.B @ u0
        xs.append(x.copy())
        v_prev = r.v
    return np.array(xs), np.array(us), results
