"""Seeded synthetic problem generators for linear-quadratic MPC (problem data only).

This module builds the data of the sparse linear-quadratic MPC problem (the paper's
Section 2, eqn. (sparse)): the dynamics A, B, the weights Q, R, Q_f, the bounds and the
initial state. It holds none of the method's arithmetic (no state elimination, no
interior-point step); both the HIP library's tests and the CPU oracle take their inputs
from here.

Workloads are explicit-Euler finite-difference heat equations with boundary or distributed
actuators, the family of the paper's Section 5 (a PDE temperature-control problem whose
states are interior grid temperatures and whose inputs act through the boundary).

Seeds: ``numpy.random.default_rng([config_id, instance_id])``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "LQProblem",
    "heat1d",
    "heat2d",
    "heat3d",
    "heat3d_dynamics",
    "HEAT3D_TABLE1",
    "heat1d_config",
    "batch_instances",
    "smooth_x0",
    "CONFIG_SMALL",
    "CONFIG_1D",
    "CONFIG_2D",
]


@dataclass
class LQProblem:
    """Data of eqn. (sparse).

    Arrays are float64, row-major.  ``A`` is ns x ns, ``B`` ns x nu, ``Q``/``Qf`` ns x ns,
    ``R`` nu x nu, ``xl``/``xu`` length ns, ``ul``/``uu`` length nu, ``x0`` length ns.
    ``N`` is the horizon (the paper's T).  Infinite bounds mean "no bound".  The general
    data are optional (None: absent): the cross weight ``S`` (ns x nu), the rows
    ``gl <= E x_t + F u_t <= gu`` (``E`` nc x ns, ``F`` nc x nu, ``gl``/``gu`` length nc), the
    disturbance ``w`` (N x ns, w_t of eqn. (dyn)) and the stabilising feedback ``Kfb``
    (nu x ns) of eqn. (K_constraint), u_t = Kfb x_t + v_t.
    """

    A: np.ndarray
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    Qf: np.ndarray
    xl: np.ndarray
    xu: np.ndarray
    ul: np.ndarray
    uu: np.ndarray
    x0: np.ndarray
    N: int
    name: str = ""
    meta: dict = field(default_factory=dict)
    S: np.ndarray | None = None
    E: np.ndarray | None = None
    F: np.ndarray | None = None
    gl: np.ndarray | None = None
    gu: np.ndarray | None = None
    w: np.ndarray | None = None
    Kfb: np.ndarray | None = None

    @property
    def general(self) -> bool:
        return any(a is not None for a in (self.S, self.E, self.F, self.w, self.Kfb))

    @property
    def nc(self) -> int:
        return 0 if self.E is None else int(self.E.shape[0])

    @property
    def ns(self) -> int:
        return int(self.A.shape[0])

    @property
    def nu(self) -> int:
        return int(self.B.shape[1])

    @property
    def n(self) -> int:
        return self.nu * self.N

    def with_x0(self, x0) -> "LQProblem":
        return LQProblem(self.A, self.B, self.Q, self.R, self.Qf, self.xl, self.xu, self.ul,
                         self.uu, np.ascontiguousarray(x0, dtype=np.float64), self.N,
                         self.name, dict(self.meta), self.S, self.E, self.F, self.gl, self.gu,
                         self.w, self.Kfb)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def heat1d_dynamics(ns: int, nu: int, r: float = 0.25, amp: float = 0.1):
    """1-D explicit-Euler heat step with zero Dirichlet ends and Gaussian-bump actuators.

    A = tridiag(r, 1 - 2r, r); B[i, j] = amp * exp(-0.5 ((i - c_j) / w)^2) with
    c_j = (j + 1/2) ns / nu - 1/2 and w = ns / (4 nu).
    """
    A = np.zeros((ns, ns))
    idx = np.arange(ns)
    A[idx, idx] = 1.0 - 2.0 * r
    A[idx[1:], idx[:-1]] = r
    A[idx[:-1], idx[1:]] = r
    c = (np.arange(nu) + 0.5) * ns / nu - 0.5
    w = ns / (4.0 * nu)
    B = amp * np.exp(-0.5 * ((idx[:, None] - c[None, :]) / w) ** 2)
    return _f64(A), _f64(B)


def heat1d(ns: int, nu: int, N: int, seed=(0, 0), *, r: float = 0.25, amp: float = 0.1,
           q: float = 1.0, rw: float = 1e-2, xb: float = 0.5, ub: float = 1.0,
           x0_range=(-0.4, 0.4), xu=None, xl=None, name: str = "") -> LQProblem:
    """1-D heat problem: Q = q I, R = rw I, Q_f = Q, |x| <= xb, |u| <= ub, x0 ~ U(x0_range)."""
    A, B = heat1d_dynamics(ns, nu, r, amp)
    rng = np.random.default_rng(list(seed))
    x0 = rng.uniform(x0_range[0], x0_range[1], size=ns)
    xu_v = np.full(ns, xb if xu is None else xu)
    xl_v = np.full(ns, -xb if xl is None else xl)
    Q = q * np.eye(ns)
    return LQProblem(A=A, B=B, Q=_f64(Q), R=_f64(rw * np.eye(nu)), Qf=_f64(Q),
                     xl=_f64(xl_v), xu=_f64(xu_v), ul=_f64(np.full(nu, -ub)),
                     uu=_f64(np.full(nu, ub)), x0=_f64(x0), N=int(N),
                     name=name or f"heat1d_ns{ns}_nu{nu}_N{N}",
                     meta={"seed": list(seed)})


def heat2d_dynamics(g: int, nu_per_edge: int = 5, r: float = 0.2):
    """2-D 5-point explicit heat step on a g x g interior grid with boundary actuators.

    Each of the 4 edges is cut into ``nu_per_edge`` equal segments; an actuator sets the
    Dirichlet value of one segment, so B[p, i] = r for every interior node p next to a
    boundary node of segment i (corner nodes touch two edges).
    """
    ns = g * g
    A = np.zeros((ns, ns))

    def node(ix, iy):
        return ix * g + iy

    for ix in range(g):
        for iy in range(g):
            p = node(ix, iy)
            A[p, p] = 1.0 - 4.0 * r
            for jx, jy in ((ix - 1, iy), (ix + 1, iy), (ix, iy - 1), (ix, iy + 1)):
                if 0 <= jx < g and 0 <= jy < g:
                    A[p, node(jx, jy)] = r
    if g % nu_per_edge:
        raise ValueError("grid size must be a multiple of the segments per edge")
    seg = g // nu_per_edge
    nu = 4 * nu_per_edge
    B = np.zeros((ns, nu))
    for k in range(g):
        s = k // seg
        B[node(0, k), 0 * nu_per_edge + s] += r          # edge x = 0
        B[node(g - 1, k), 1 * nu_per_edge + s] += r      # edge x = L
        B[node(k, 0), 2 * nu_per_edge + s] += r          # edge y = 0
        B[node(k, g - 1), 3 * nu_per_edge + s] += r      # edge y = L
    return _f64(A), _f64(B)


def heat2d(g: int = 70, nu_per_edge: int = 5, N: int = 100, seed=(2, 0), *, r: float = 0.2,
           q: float = 1.0, rw: float = 1e-2, xb: float = 0.5, ub: float = 1.0,
           x0_range=(-0.4, 0.4), name: str = "") -> LQProblem:
    A, B = heat2d_dynamics(g, nu_per_edge, r)
    ns, nu = B.shape
    rng = np.random.default_rng(list(seed))
    x0 = rng.uniform(x0_range[0], x0_range[1], size=ns)
    Q = q * np.eye(ns)
    return LQProblem(A=A, B=B, Q=_f64(Q), R=_f64(rw * np.eye(nu)), Qf=_f64(Q),
                     xl=_f64(np.full(ns, -xb)), xu=_f64(np.full(ns, xb)),
                     ul=_f64(np.full(nu, -ub)), uu=_f64(np.full(nu, ub)), x0=_f64(x0),
                     N=int(N), name=name or f"heat2d_{g}x{g}_nu{nu}_N{N}",
                     meta={"seed": list(seed)})


# Table 1 of the paper: the copper cube of the 3-D temperature-control problem (Section 5).
HEAT3D_TABLE1 = dict(dt=0.1, dw=0.02, rho=8960.0, cp=386.0, k=400.0, xl=200.0, xu=550.0,
                     ul=300.0, uu=500.0, xhat=300.0)


def heat3d_dynamics(m: int, dt: float = 0.1, dw: float = 0.02, rho: float = 8960.0,
                    cp: float = 386.0, k: float = 400.0):
    """3-D 7-point explicit-Euler heat step on the m^3 interior nodes of a cube (Section 5,
    eqn. (3DPDE), Table 1): x+ = x + r (sum of the 6 neighbours - 6 x), r = k dt / (rho cp dw^2).

    The 6 faces are the inputs (Dirichlet values, not states): a neighbour that lies on face
    i contributes r u_i, so B[p, i] = r for each such neighbour (nodes next to an edge or a
    corner touch 2 or 3 faces).  Faces: 0/1 x = 0/L, 2/3 y = 0/L, 4/5 z = 0/L.
    """
    r = k * dt / (rho * cp * dw * dw)
    ns = m * m * m
    A = np.zeros((ns, ns))
    B = np.zeros((ns, 6))

    def node(ix, iy, iz):
        return (ix * m + iy) * m + iz

    for ix in range(m):
        for iy in range(m):
            for iz in range(m):
                p = node(ix, iy, iz)
                A[p, p] = 1.0 - 6.0 * r
                c = (ix, iy, iz)
                for axis in range(3):
                    for step, face in ((-1, 2 * axis), (1, 2 * axis + 1)):
                        nb = list(c)
                        nb[axis] += step
                        if 0 <= nb[axis] < m:
                            A[p, node(*nb)] = r
                        else:
                            B[p, face] += r
    return _f64(A), _f64(B)


def heat3d(m: int, N: int, *, setpoint: float = 400.0, name: str = "", **table) -> LQProblem:
    """The paper's 3-D cube (m interior nodes per dimension, horizon N = the paper's T) with
    Table 1's constants, written in deviations from a uniform set point d: x - d, u - d.

    The paper's set point is not given; a uniform d is a steady state of the dynamics with every
    face at d (A 1 + B 1 = 1), so in deviation form the problem has the library's pure
    quadratic cost: Q = q I (q = 10 dw^2), R = r I (r = dw^2 / 10) penalise the state's
    distance to d and the inputs' distance to d.  Bounds and the initial state are Table 1's
    less d.
    """
    c = dict(HEAT3D_TABLE1)
    c.update(table)
    A, B = heat3d_dynamics(m, c["dt"], c["dw"], c["rho"], c["cp"], c["k"])
    ns, nu = B.shape
    q, rw = 10.0 * c["dw"] ** 2, 0.1 * c["dw"] ** 2
    Q = q * np.eye(ns)
    return LQProblem(A=A, B=B, Q=_f64(Q), R=_f64(rw * np.eye(nu)), Qf=_f64(Q),
                     xl=_f64(np.full(ns, c["xl"] - setpoint)),
                     xu=_f64(np.full(ns, c["xu"] - setpoint)),
                     ul=_f64(np.full(nu, c["ul"] - setpoint)),
                     uu=_f64(np.full(nu, c["uu"] - setpoint)),
                     x0=_f64(np.full(ns, c["xhat"] - setpoint)), N=int(N),
                     name=name or f"heat3d_m{m}_T{N}", meta={"setpoint": setpoint})


# Named workloads (sizes of the benchmark and parity cases).
def general_random(ns: int, nu: int, nc: int, N: int, seed: int, *, rho: float = 1.05,
                   bound_x: float = 0.6, bound_u: float = 1.0, bound_g: float = 0.25,
                   w_scale: float = 0.02, x0_scale: float = 0.3, feedback: bool = True,
                   cross: bool = True) -> LQProblem:
    """A random instance of eqn. (sparse) with every kind of data: an A of spectral radius
    rho (above 1: open-loop unstable), a joint weight [[Q, S], [S', R]] > 0, nc rows
    gl <= E x + F u <= gu, a disturbance w_t and (feedback) the stabilising gain of the
    infinite-horizon LQR of (A, B, Q, R) as Kfb, so that A + B Kfb is stable (the reason
    eqn. (K_constraint) introduces it)."""
    import scipy.linalg as sla
    rng = np.random.default_rng([77, ns, nu, nc, N, seed])
    A = rng.normal(size=(ns, ns))
    A *= rho / max(1e-12, np.max(np.abs(np.linalg.eigvals(A))))
    B = rng.normal(size=(ns, nu))
    M = rng.normal(size=(ns + nu, ns + nu))
    Wj = M @ M.T / (ns + nu) + 0.3 * np.eye(ns + nu)
    Q, R = Wj[:ns, :ns].copy(), Wj[ns:, ns:].copy()
    S = Wj[:ns, ns:].copy() if cross else None
    Kfb = None
    if feedback:
        P = sla.solve_discrete_are(A, B, Q, R)
        Kfb = -np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
    E = rng.normal(size=(nc, ns)) / np.sqrt(ns) if nc > 0 else None
    F = rng.normal(size=(nc, nu)) / np.sqrt(nu) if nc > 0 else None
    gl = np.full(nc, -bound_g) if nc > 0 else None
    gu = np.full(nc, bound_g) if nc > 0 else None
    w = w_scale * rng.normal(size=(N, ns)) if w_scale > 0 else None
    x0 = rng.uniform(-x0_scale, x0_scale, ns)
    return LQProblem(A=_f64(A), B=_f64(B), Q=_f64(Q), R=_f64(R), Qf=_f64(2.0 * Q),
                     xl=np.full(ns, -bound_x), xu=np.full(ns, bound_x), ul=np.full(nu, -bound_u),
                     uu=np.full(nu, bound_u), x0=_f64(x0), N=N,
                     name=f"general_{ns}_{nu}_{nc}_{N}_{seed}",
                     S=None if S is None else _f64(S), E=None if E is None else _f64(E),
                     F=None if F is None else _f64(F), gl=gl, gu=gu,
                     w=None if w is None else _f64(w), Kfb=None if Kfb is None else _f64(Kfb))


def heat1d_general(ns: int, nu: int, N: int, seed=(6, 0), *, kgain: float = 0.5,
                   cross: float = 0.02, src: float = 0.004, gbound: float = 0.15) -> LQProblem:
    """The 1-D heat workload with the general data: a proportional feedback Kfb =
    -kgain B' (each actuator pulls against the temperature under it; A + B Kfb stays
    stable), a small cross weight S = cross B, a constant heat source w_t = src * (the sum of
    the actuator bumps, normalised), and two stage rows: the total actuation
    |sum_j u_j| <= gbound (E = 0, F = 1') and the mean temperature |mean(x)| <= gbound / 4
    (E = 1'/ns, F = 0)."""
    p = heat1d(ns, nu, N, seed=seed, xu=0.3, x0_range=(-0.25, 0.25))
    B = p.B
    bump = B.sum(axis=1)
    w = np.tile(src * bump / max(1e-12, np.max(bump)), (N, 1))
    E = np.vstack([np.zeros(ns), np.full(ns, 1.0 / ns)])
    F = np.vstack([np.ones(nu), np.zeros(nu)])
    g = np.array([gbound, gbound / 4.0])
    return LQProblem(A=p.A, B=B, Q=p.Q, R=p.R, Qf=p.Qf, xl=p.xl, xu=p.xu, ul=p.ul, uu=p.uu,
                     x0=p.x0, N=N, name=f"heat1d_general_{ns}_{nu}_{N}", S=_f64(cross * B),
                     E=_f64(E), F=_f64(F), gl=_f64(-g), gu=_f64(g), w=_f64(w),
                     Kfb=_f64(-kgain * B.T))


CONFIG_SMALL = dict(ns=50, nu=5, N=10)       # K is 50 x 50, 500 state rows
CONFIG_1D = dict(ns=1000, nu=10, N=50)       # K is 500 x 500, 50,000 state rows
CONFIG_2D = dict(g=70, nu_per_edge=5, N=100)  # K is 2000 x 2000, 490,000 state rows


def heat1d_config(which: str = "1d", instance: int = 0, **kw) -> LQProblem:
    """The named 1-D workloads: 'small' (config id 0) and '1d' (config id 1)."""
    if which == "small":
        return heat1d(**CONFIG_SMALL, seed=(0, instance), **kw)
    if which == "1d":
        return heat1d(**CONFIG_1D, seed=(1, instance), **kw)
    raise ValueError(which)


def batch_instances(count: int = 512, seed: int = 3, ns_range=(100, 2000), nu_range=(2, 16),
                    N_range=(16, 64)) -> list:
    """Independent 1-D heat instances of uneven size for batched solves.

    ns ~ U{ns_range}, nu ~ U{nu_range}, N ~ U{N_range}, x^u = -x^l ~ U(0.45, 0.6),
    u^u = -u^l ~ U(0.5, 1.5), x0 ~ U(-0.4, 0.4); instance i uses default_rng([seed, i]).
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
        nu = int(rng.integers(nu_range[0], nu_range[1] + 1))
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        xb = float(rng.uniform(0.45, 0.6))
        ub = float(rng.uniform(0.5, 1.5))
        A, B = heat1d_dynamics(ns, nu)
        x0 = rng.uniform(-0.4, 0.4, size=ns)
        Q = np.eye(ns)
        out.append(LQProblem(A=A, B=B, Q=Q, R=1e-2 * np.eye(nu), Qf=Q.copy(),
                             xl=np.full(ns, -xb), xu=np.full(ns, xb), ul=np.full(nu, -ub),
                             uu=np.full(nu, ub), x0=_f64(x0), N=N,
                             name=f"batch{seed}_{i}", meta={"seed": [seed, i]}))
    return out


def smooth_x0(ns: int, count: int, seed: int = 4, amp: float = 0.4, modes: int = 8) -> np.ndarray:
    """Smooth random initial temperature fields, one per row (count x ns).

    f = sum_k a_k sin(k pi (i + 1) / (ns + 1)), a_k ~ N(0, k^-2), k = 1..modes;
    x0 = rho * amp * f / max|f| with rho ~ U(0, 1].
    """
    rng = np.random.default_rng([seed, ns])
    i = np.arange(ns)
    k = np.arange(1, modes + 1)
    basis = np.sin(np.outer(k, (i + 1)) * np.pi / (ns + 1))      # modes x ns
    a = rng.normal(size=(count, modes)) / k[None, :]
    f = a @ basis
    rho = 1.0 - rng.uniform(0.0, 1.0, size=count)                  # (0, 1]
    scale = np.max(np.abs(f), axis=1)
    scale[scale == 0] = 1.0
    return _f64(rho[:, None] * amp * f / scale[:, None])


# ---------------------------------------------------------------- surrogate inputs
def mlp_widths(ns: int, n_out: int, hidden: int = 1024, depth: int = 4) -> list:
    return [ns] + [hidden] * depth + [n_out]


def mlp_init(widths, seed: int = 5) -> np.ndarray:
    """Packed float32 initial parameters W_1, b_1, ..., W_L, b_L (W_l row-major, d_l x d_(l-1)),
    every entry ~ U(-1/sqrt(d_(l-1)), 1/sqrt(d_(l-1)))."""
    rng = np.random.default_rng([seed, len(widths)])
    parts = []
    for l in range(1, len(widths)):
        bound = 1.0 / np.sqrt(widths[l - 1])
        parts.append(rng.uniform(-bound, bound, size=widths[l] * widths[l - 1]))
        parts.append(rng.uniform(-bound, bound, size=widths[l]))
    return np.concatenate(parts).astype(np.float32)


def unpack_params(flat, widths) -> list:
    """[(W_l, b_l)] float64 views of a packed parameter vector."""
    out, off = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for l in range(1, len(widths)):
        nW = widths[l] * widths[l - 1]
        W = flat[off:off + nW].reshape(widths[l], widths[l - 1])
        off += nW
        b = flat[off:off + widths[l]]
        off += widths[l]
        out.append((W, b))
    return out


def shuffle_order(count: int, epochs: int, seed: int = 6) -> np.ndarray:
    """Row order of each training epoch (epochs x count, int32)."""
    rng = np.random.default_rng([seed, count])
    return np.concatenate([rng.permutation(count) for _ in range(epochs)]).astype(np.int32)
