"""Plain FP64 CPU oracle of the learned surrogate policy x0 -> u and of its judge.

TEST INFRASTRUCTURE ONLY (same rule as ``oracle.condensed_ipm``): only the test suite,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import it, and it
imports nothing from the HIP library or its binding.

The surrogate is a library extension, not part of the paper: a multilayer perceptron maps
an initial state x0 to the whole control sequence u = (u_0, ..., u_{N-1}) of the
condensed QP of Section 2, and the interior-point method of Section 3 judges every answer
and replaces the ones it cannot certify.  What is computed here, written out from the
definitions:

Network (widths d_0 = ns, d_1..d_L = hidden, d_{L+1} = nu N; layer l has W_l of shape
d_l x d_{l-1} and b_l of length d_l):
    a_0 = r(X)
    z_l = a_{l-1} r(W_l)' + b_l,   a_l = r(gelu(z_l))            l = 1..L
    y   = a_L r(W_{L+1})' + b_{L+1}                              (not rounded)
    u   = clip(y, ul, uu)                                        (inference only)
gelu(x) = x Phi(x) with Phi the standard normal distribution function (exact form).
r() rounds to bfloat16 (round to nearest, ties to even) in "bf16" mode and is the identity
in "fp32" mode; products of rounded values are exact here and sums are float64, so the
oracle isolates the rounding points and leaves only accumulation order to the tolerance.

Loss: mean squared error over the rows and the d_{L+1} outputs, L = mean((y - U*)^2), on
the unclipped output.  Its gradient by the chain rule, with the same rounding points as
the forward pass:
    g_{L+1} = r(2 (y - U*) / (M d_{L+1}))
    dW_l = g_l' a_{l-1},   db_l = column sums of g_l
    g_l  = r((g_{l+1} r(W_{l+1})) * gelu'(z_l))                 l = L..1

AdamW (Loshchilov and Hutter, decoupled weight decay), step t = 1, 2, ...:
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    w = w - lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd w)
with wd applied to the weight matrices and not to the biases.

Judge (float64): for a query x0 and an answer u,
    violation = max(0, x - xu, xl - x, u - uu, ul - u) over the simulated states
                x_1..x_N (eqn. (dyn)) and the controls (infinite bounds ignored);
    f(u)      = objective of eqn. (sparse) by simulation (1/2 convention);
    LB(x0)    = h0 - 1/2 h' H^-1 h, the dual function at lambda = 0, i.e. the minimum of
                the unconstrained QP, so LB <= f* <= f(u) (weak duality);
    accept    iff violation <= 1e-4 and (f(u) - LB) / |LB| <= 1e-3.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.special import erf

from .condensed_ipm import reduce_problem, simulate, sparse_objective

VIOLATION_TOL = 1e-4
GAP_TOL = 1e-3


# ------------------------------------------------------------------ rounding and GELU
def bf16_round(x) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64.

    A bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of a float32.
    Values are first rounded to float32 (exactly representable ones are unchanged), then
    the low 16 bits of the float32 pattern are rounded off."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    finite = np.isfinite(f)
    out = np.where(finite, rounded, bits & np.uint64(0xFFFF0000)).astype(np.uint32)
    return out.view(np.float32).astype(np.float64)


def rounder(mode: str):
    if mode == "bf16":
        return bf16_round
    if mode == "fp32":
        return lambda a: np.asarray(a, dtype=np.float64)
    raise ValueError(mode)


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx x Phi(x) = Phi(x) + x phi(x)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(
        2.0 * math.pi)


# ------------------------------------------------------------------ network
def widths(ns: int, n_out: int, hidden: int = 1024, depth: int = 4):
    return [ns] + [hidden] * depth + [n_out]


def param_count(w) -> int:
    return int(sum(w[i + 1] * w[i] + w[i + 1] for i in range(len(w) - 1)))


def forward(params, X, mode="bf16"):
    """params: list of (W, b); X: M x d_0.  Returns (y, cache) with cache = (a list, z list)."""
    r = rounder(mode)
    a = [r(X)]
    zs = []
    L = len(params) - 1
    for l, (W, b) in enumerate(params):
        z = a[-1] @ r(W).T + b
        if l < L:
            zs.append(z)
            a.append(r(gelu(z)))
        else:
            return z, (a, zs)


def loss(y, U):
    return float(np.mean((y - U) ** 2))


def backward(params, cache, y, U, mode="bf16"):
    """Gradients [(dW, db)] of the MSE loss, with the rounding points of the forward pass."""
    r = rounder(mode)
    a, zs = cache
    M, nout = y.shape
    g = r(2.0 * (y - U) / (M * nout))
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        grads[l] = (g.T @ a[l], g.sum(axis=0))
        if l > 0:
            g = r((g @ r(params[l][0])) * gelu_grad(zs[l - 1]))
    return grads


def adamw_step(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update (returns new w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v


def predict(params, X, ul, uu, mode="bf16"):
    """Clipped controls for a batch of x0 (ul, uu of length n_out)."""
    y, _ = forward(params, X, mode)
    return np.clip(y, ul, uu)


# ------------------------------------------------------------------ judge
def violation(prob, u) -> float:
    x = simulate(prob, u)
    N, nu = int(prob.N), prob.B.shape[1]
    xu, xl = np.tile(prob.xu, N), np.tile(prob.xl, N)
    uu, ul = np.tile(prob.uu, N), np.tile(prob.ul, N)
    parts = [0.0]
    for hi, lo, val in ((xu, xl, x), (uu, ul, u)):
        with np.errstate(invalid="ignore"):
            up = np.where(np.isinf(hi), -np.inf, val - hi)
            dn = np.where(np.isinf(lo), -np.inf, lo - val)
        parts += [float(np.max(up, initial=-np.inf)), float(np.max(dn, initial=-np.inf))]
    return max(parts)


def lower_bound(red) -> float:
    """h0 - 1/2 h' H^-1 h by a Cholesky factorisation of H (the lambda = 0 dual value)."""
    c = sla.cho_factor(red.H, lower=True)
    return float(red.h0 - 0.5 * red.h @ sla.cho_solve(c, red.h))


def judge(prob, u, red=None):
    """(accept, violation, f, LB, certified relative gap) of an answer u for prob.x0."""
    red = reduce_problem(prob) if red is None else red
    vio = violation(prob, u)
    f = sparse_objective(prob, u)
    lb = lower_bound(red)
    gap = (f - lb) / abs(lb) if lb != 0.0 else (0.0 if f == lb else math.inf)
    return (vio <= VIOLATION_TOL and gap <= GAP_TOL), vio, f, lb, gap
