"""Independent checks that pin the CPU oracle (none of them shares the oracle's algorithm).

* ``riccati``            -- finite-horizon LQR by the backward Riccati recursion: the exact
                            minimiser when no bound is active.
* ``scalar_clamp``       -- closed form for ns = nu = N = 1 with bounds.
* ``active_set``         -- exhaustive active-set enumeration of the dense QP (tiny sizes).
* ``full_space_step``    -- the primal-dual Newton step of the *sparse* problem (states kept
                            as variables, dynamics as equality constraints), assembled
                            directly from A, B, Q, R and solved densely.  Eliminating the
                            dynamics exactly leaves the condensed step unchanged, so the two
                            must agree.
* ``augmented_step``     -- the 3 x 3 block system of eqn. (aug_KKT) solved densely.
"""
from __future__ import annotations

import itertools

import numpy as np


def riccati(prob):
    """u* and f* of the unconstrained problem (1/2 convention).

    P_N = Q_f, K_t = (R + B'P_{t+1}B)^-1 B'P_{t+1}A, P_t = Q + A'P_{t+1}(A - B K_t),
    u_t = -K_t x_t, f* = 1/2 x0' P_0 x0.
    """
    A, B, Q, R, Qf, N = prob.A, prob.B, prob.Q, prob.R, prob.Qf, int(prob.N)
    P = Qf.copy()
    gains = [None] * N
    for t in range(N - 1, -1, -1):
        K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        gains[t] = K
        P = Q + A.T @ P @ (A - B @ K)
        P = 0.5 * (P + P.T)
    x = prob.x0.copy()
    u = []
    for t in range(N):
        ut = -gains[t] @ x
        u.append(ut)
        x = A @ x + B @ ut
    return np.concatenate(u), float(0.5 * prob.x0 @ P @ prob.x0)


def scalar_clamp(a, b, q, qf, r, x0, xl, xu, ul, uu):
    """ns = nu = N = 1, b > 0: f(u) = 1/2 q x0^2 + 1/2 r u^2 + 1/2 qf (a x0 + b u)^2 is a convex
    parabola in u, so the bounded minimiser is the clamp of the free one into the interval
    where u and x1 = a x0 + b u both satisfy their bounds."""
    assert b > 0
    u_free = -qf * a * b * x0 / (r + qf * b * b)
    lo = max(ul, (xl - a * x0) / b)
    hi = min(uu, (xu - a * x0) / b)
    u = min(max(u_free, lo), hi)
    f = 0.5 * q * x0 * x0 + 0.5 * r * u * u + 0.5 * qf * (a * x0 + b * u) ** 2
    return u, f


def active_set(H, h, J, d, pairs):
    """Exact minimiser of 1/2 v'Hv + h'v s.t. Jv <= d by enumerating active sets.

    ``pairs`` lists, for every bounded quantity, its (upper row, lower row) indices in J
    (either may be None).  Each quantity is free, at its upper or at its lower bound.
    Returns (v, multipliers) of the unique primal-feasible, dual-feasible candidate.
    """
    n = H.shape[0]
    best = None
    for choice in itertools.product((0, 1, 2), repeat=len(pairs)):
        act = []
        for (up, lo), c in zip(pairs, choice):
            if c == 1:
                if up is None:
                    break
                act.append(up)
            elif c == 2:
                if lo is None:
                    break
                act.append(lo)
        else:
            if len(act) > n:
                continue
            JA = J[act]
            k = len(act)
            if k and np.linalg.matrix_rank(JA, tol=1e-9 * max(1.0, np.abs(JA).max())) < k:
                continue      # dependent active rows: covered by a smaller active set
            M = np.zeros((n + k, n + k))
            M[:n, :n] = H
            M[:n, n:] = JA.T
            M[n:, :n] = JA
            rhs = np.concatenate([-h, d[act]])
            try:
                sol = np.linalg.solve(M, rhs)
            except np.linalg.LinAlgError:
                continue
            v, lamA = sol[:n], sol[n:]
            scale = 1.0 + np.max(np.abs(d))
            if np.all(J @ v <= d + 1e-10 * scale) and np.all(lamA >= -1e-10):
                lam = np.zeros(J.shape[0])
                lam[act] = lamA
                if best is None:
                    best = (v, lam)
                else:
                    assert np.allclose(best[0], v, atol=1e-8), "two optimal active sets disagree"
    if best is None:
        raise RuntimeError("no optimal active set found")
    return best


def sparse_rows(prob):
    """Inequality rows of eqn. (sparse) over y = [u_0..u_{N-1}, x_1..x_N], in the order
    x <= xu (t = 1..N), -x <= -xl, u <= uu, -u <= -ul, rows with infinite bounds dropped."""
    ns, nu, N = prob.A.shape[0], prob.B.shape[1], int(prob.N)
    nuN, nsN = nu * N, ns * N
    ny = nuN + nsN
    rows, rhs = [], []
    for sign, bound, off, cnt, vec in ((1, prob.xu, nuN, nsN, prob.xu),
                                       (-1, prob.xl, nuN, nsN, prob.xl),
                                       (1, prob.uu, 0, nuN, prob.uu),
                                       (-1, prob.ul, 0, nuN, prob.ul)):
        per = len(vec)
        for k in range(cnt):
            b = vec[k % per]
            if not np.isfinite(b):
                continue
            row = np.zeros(ny)
            row[off + k] = sign
            rows.append(row)
            rhs.append(sign * b)
    return np.array(rows), np.array(rhs)


def full_space_step(prob, u, s, lam, z, mu):
    """Primal-dual Newton step of the sparse problem at y = (u, x(u)) with nu = 0.

    Unknowns (p_y, p_nu, p_s, p_lambda); returns (p_u, p_s, p_lambda, p_z) where
    p_z = mu/s - z - (z/s) p_s is the Newton step of S Z 1 = mu 1.
    """
    A, B, Q, R, Qf = prob.A, prob.B, prob.Q, prob.R, prob.Qf
    ns, nu, N = A.shape[0], B.shape[1], int(prob.N)
    nuN, nsN = nu * N, ns * N
    ny = nuN + nsN
    # states by simulation
    x = prob.x0.copy()
    xs = []
    for t in range(N):
        x = A @ x + B @ u[t * nu:(t + 1) * nu]
        xs.append(x)
    y = np.concatenate([u] + xs)
    # Hessian of the objective
    P = np.zeros((ny, ny))
    for t in range(N):
        P[t * nu:(t + 1) * nu, t * nu:(t + 1) * nu] = R
    for t in range(1, N + 1):
        o = nuN + (t - 1) * ns
        P[o:o + ns, o:o + ns] = Qf if t == N else Q
    # dynamics rows: x_{t+1} - A x_t - B u_t = (A x0 if t == 0 else 0)
    E = np.zeros((nsN, ny))
    e = np.zeros(nsN)
    for t in range(N):
        r = t * ns
        E[r:r + ns, nuN + t * ns:nuN + (t + 1) * ns] = np.eye(ns)
        E[r:r + ns, t * nu:(t + 1) * nu] = -B
        if t == 0:
            e[r:r + ns] = A @ prob.x0
        else:
            E[r:r + ns, nuN + (t - 1) * ns:nuN + t * ns] = -A
    C, ds = sparse_rows(prob)
    m = C.shape[0]
    sigma = z / s
    nu_mult = np.zeros(nsN)
    g1 = P @ y + E.T @ nu_mult + C.T @ lam
    g2 = E @ y - e
    g3 = lam - mu / s
    g4 = C @ y - ds + s
    size = ny + nsN + 2 * m
    M = np.zeros((size, size))
    o1, o2, o3 = ny, ny + nsN, ny + nsN + m
    M[:ny, :ny] = P
    M[:ny, o1:o2] = E.T
    M[:ny, o3:] = C.T
    M[o1:o2, :ny] = E
    M[o2:o3, o2:o3] = np.diag(sigma)
    M[o2:o3, o3:] = np.eye(m)
    M[o3:, :ny] = C
    M[o3:, o2:o3] = np.eye(m)
    sol = np.linalg.solve(M, -np.concatenate([g1, g2, g3, g4]))
    pu = sol[:nuN]
    ps = sol[o2:o3]
    plam = sol[o3:]
    pz = mu / s - z - sigma * ps
    return pu, ps, plam, pz


def augmented_step(H, h, J, d, v, s, lam, mu, z):
    """Eqn. (aug_KKT) solved densely for (p_v, p_s, p_lambda)."""
    n, m = H.shape[0], J.shape[0]
    sigma = z / s
    r1 = H @ v + h + J.T @ lam
    r2 = lam - mu / s
    r3 = J @ v - d + s
    M = np.zeros((n + 2 * m, n + 2 * m))
    M[:n, :n] = H
    M[:n, n + m:] = J.T
    M[n:n + m, n:n + m] = np.diag(sigma)
    M[n:n + m, n + m:] = np.eye(m)
    M[n + m:, :n] = J
    M[n + m:, n:n + m] = np.eye(m)
    sol = np.linalg.solve(M, -np.concatenate([r1, r2, r3]))
    return sol[:n], sol[n:n + m], sol[n + m:]


# ---------------------------------------------------------------- general data (S, E, F, w, K)
# Written from eqn. (sparse) directly, with the states as variables; they share nothing with
# the oracle's elimination.

def simulate_general(prob, v):
    """Trajectory under u_t = K x_t + v_t (eqn. (K_constraint)) and
    x_{t+1} = A x_t + B u_t + w_t (eqn. (dyn)): states x_0..x_N (rows) and inputs u_0..u_{N-1}."""
    ns, nu, N = prob.A.shape[0], prob.B.shape[1], int(prob.N)
    K = np.zeros((nu, ns)) if prob.Kfb is None else prob.Kfb
    xs = [np.array(prob.x0, dtype=np.float64)]
    us = []
    for t in range(N):
        u = K @ xs[-1] + v[t * nu:(t + 1) * nu]
        us.append(u)
        x = prob.A @ xs[-1] + prob.B @ u
        if prob.w is not None:
            x = x + prob.w[t]
        xs.append(x)
    return np.array(xs), np.array(us)


def objective_general(prob, xs, us):
    """Objective of eqn. (sparse), 1/2 convention: sum_t 1/2 [x;u]'[[Q, S], [S', R]][x;u] +
    1/2 x_N' Q_f x_N."""
    S = np.zeros((prob.A.shape[0], prob.B.shape[1])) if prob.S is None else prob.S
    f = 0.0
    for t in range(int(prob.N)):
        x, u = xs[t], us[t]
        f += 0.5 * x @ prob.Q @ x + x @ S @ u + 0.5 * u @ prob.R @ u
    return float(f + 0.5 * xs[-1] @ prob.Qf @ xs[-1])


def constraint_values(prob, xs, us):
    """Left sides minus right sides of every inequality of eqn. (sparse), by kind:
    {0: x - xu, 1: xl - x (t = 1..N), 2: u - uu, 3: ul - u, 4: Ex + Fu - gu,
    5: gl - (Ex + Fu) (t = 0..N-1)}, each stacked over t."""
    N = int(prob.N)
    X = xs[1:]
    out = {0: (X - prob.xu).ravel(), 1: (prob.xl - X).ravel(), 2: (us - prob.uu).ravel(),
           3: (prob.ul - us).ravel()}
    if prob.E is not None:
        g = np.array([prob.E @ xs[t] + prob.F @ us[t] for t in range(N)])
        out[4] = (g - prob.gu).ravel()
        out[5] = (prob.gl - g).ravel()
    return out


def riccati_cross(prob):
    """Unconstrained minimiser with a cross weight (no feedback, no disturbance): the
    backward recursion P_N = Q_f, L_t = (R + B'P B)^-1 (B'P A + S'),
    P_t = Q + A'P A - (A'P B + S) L_t, u_t = -L_t x_t, f* = 1/2 x0' P_0 x0."""
    A, B, Q, R, Qf, N = prob.A, prob.B, prob.Q, prob.R, prob.Qf, int(prob.N)
    S = prob.S
    P = Qf.copy()
    gains = [None] * N
    for t in range(N - 1, -1, -1):
        L = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A + S.T)
        gains[t] = L
        P = Q + A.T @ P @ A - (A.T @ P @ B + S) @ L
        P = 0.5 * (P + P.T)
    x = prob.x0.copy()
    u = []
    for t in range(N):
        ut = -gains[t] @ x
        u.append(ut)
        x = A @ x + B @ ut
    return np.concatenate(u), float(0.5 * prob.x0 @ P @ prob.x0)


def sparse_active_set(prob):
    """Exact minimiser of eqn. (sparse) in its own variables y = [u_0..u_{N-1}, x_1..x_N]
    (the dynamics as equality constraints, the feedback gain plays no part) by enumerating
    which bound of every bounded quantity (x_t,i, u_t,j, (E x_t + F u_t)_k) is active.
    Returns (u*, f*).  Tiny sizes only (3^quantities equality-constrained solves)."""
    A, B, Q, R, Qf = prob.A, prob.B, prob.Q, prob.R, prob.Qf
    ns, nu, N = A.shape[0], B.shape[1], int(prob.N)
    S = np.zeros((ns, nu)) if prob.S is None else prob.S
    w = np.zeros((N, ns)) if prob.w is None else prob.w
    x0 = prob.x0
    nU, nX = nu * N, ns * N
    ny = nU + nX
    ui = lambda t: slice(t * nu, (t + 1) * nu)                 # noqa: E731
    xi = lambda t: slice(nU + (t - 1) * ns, nU + t * ns)       # t = 1..N  # noqa: E731
    P = np.zeros((ny, ny))
    q = np.zeros(ny)
    const = 0.5 * x0 @ Q @ x0
    for t in range(N):
        P[ui(t), ui(t)] += R
        if t == 0:
            q[ui(0)] += S.T @ x0
        else:
            P[xi(t), xi(t)] += Q
            P[xi(t), ui(t)] += S
            P[ui(t), xi(t)] += S.T
    P[xi(N), xi(N)] += Qf
    Aeq = np.zeros((nX, ny))
    beq = np.zeros(nX)
    for t in range(N):
        r = slice(t * ns, (t + 1) * ns)
        Aeq[r, xi(t + 1)] = np.eye(ns)
        Aeq[r, ui(t)] = -B
        if t == 0:
            beq[r] = A @ x0 + w[0]
        else:
            Aeq[r, xi(t)] = -A
            beq[r] = w[t]
    rows, rhs, pairs = [], [], []

    def add_pair(a, a0, lo, hi):
        """a y + a0 in [lo, hi]: rows a y <= hi - a0 and -a y <= a0 - lo."""
        up = lw = None
        if np.isfinite(hi):
            up = len(rows)
            rows.append(a)
            rhs.append(hi - a0)
        if np.isfinite(lo):
            lw = len(rows)
            rows.append(-a)
            rhs.append(a0 - lo)
        if up is not None or lw is not None:
            pairs.append((up, lw))

    for t in range(1, N + 1):
        for i in range(ns):
            a = np.zeros(ny)
            a[xi(t).start + i] = 1.0
            add_pair(a, 0.0, prob.xl[i], prob.xu[i])
    for t in range(N):
        for j in range(nu):
            a = np.zeros(ny)
            a[ui(t).start + j] = 1.0
            add_pair(a, 0.0, prob.ul[j], prob.uu[j])
    if prob.E is not None:
        for t in range(N):
            for k in range(prob.E.shape[0]):
                a = np.zeros(ny)
                a[ui(t)] = prob.F[k]
                a0 = 0.0
                if t == 0:
                    a0 = prob.E[k] @ x0
                else:
                    a[xi(t)] = prob.E[k]
                add_pair(a, a0, prob.gl[k], prob.gu[k])
    C, dC = np.array(rows), np.array(rhs)
    best = None
    for choice in itertools.product((0, 1, 2), repeat=len(pairs)):
        act = []
        for (up, lw), c in zip(pairs, choice):
            if c == 1:
                if up is None:
                    break
                act.append(up)
            elif c == 2:
                if lw is None:
                    break
                act.append(lw)
        else:
            k = len(act)
            Geq = np.vstack([Aeq, C[act]]) if k else Aeq
            if np.linalg.matrix_rank(Geq, tol=1e-9) < nX + k:
                continue      # dependent active rows: covered by a smaller active set
            M = np.zeros((ny + nX + k, ny + nX + k))
            M[:ny, :ny] = P
            M[:ny, ny:ny + nX] = Aeq.T
            M[ny:ny + nX, :ny] = Aeq
            if k:
                M[:ny, ny + nX:] = C[act].T
                M[ny + nX:, :ny] = C[act]
            b = np.concatenate([-q, beq, dC[act]])
            try:
                sol = np.linalg.solve(M, b)
            except np.linalg.LinAlgError:
                continue
            if not np.all(np.isfinite(sol)):
                continue
            y, lam = sol[:ny], sol[ny + nX:]
            scale = 1.0 + np.max(np.abs(dC))
            if (np.all(C @ y <= dC + 1e-10 * scale) and np.all(lam >= -1e-10)
                    and np.max(np.abs(Aeq @ y - beq)) <= 1e-10 * (1.0 + np.max(np.abs(beq)))):
                f = 0.5 * y @ P @ y + q @ y + const
                if best is None or f < best[1] - 1e-12:
                    best = (y[:nU].copy(), float(f))
    if best is None:
        raise RuntimeError("no optimal active set found")
    return best
