"""Pins of the surrogate oracle (oracle/surrogate.py) against facts independent of it:
a library bfloat16 conversion, the standard normal distribution, finite differences,
closed forms of AdamW, the Riccati closed form of the unconstrained LQ problem, and
hand-solvable scalar cases."""
import math

import numpy as np
import pytest
import scipy.stats
import torch

import oracle
from oracle import surrogate as S
from paper_2209_13049_amd import workloads as W
from brute_force import riccati


def test_bf16_round_known_values():
    one = 1.0
    assert S.bf16_round(one) == 1.0
    assert S.bf16_round(1 + 2.0 ** -8) == 1.0                   # tie -> even (k = 0)
    assert S.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6     # tie -> even (k = 2)
    assert S.bf16_round(1 + 2.0 ** -7) == 1 + 2.0 ** -7         # representable
    assert S.bf16_round(-2.5) == -2.5
    assert S.bf16_round(0.0) == 0.0


def test_bf16_round_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-6, 6, size=20000),
                        np.array([1e-40, -3e-39, 65504.0, 3.3e38])])
    x32 = x.astype(np.float32)
    lib = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    ours = S.bf16_round(x32.astype(np.float64))
    assert np.array_equal(lib, ours)
    # relative error bound and idempotence
    nz = np.abs(x32) > 1e-30
    assert np.all(np.abs(ours[nz] - x32[nz]) <= 2.0 ** -8 * np.abs(x32[nz]))
    assert np.array_equal(S.bf16_round(ours), ours)


def test_gelu_against_normal_cdf():
    x = np.linspace(-8, 8, 2001)
    ref = x * scipy.stats.norm.cdf(x)
    assert np.max(np.abs(S.gelu(x) - ref)) <= 1e-14
    assert np.max(np.abs(S.gelu(x) - S.gelu(-x) - x)) <= 1e-13   # x Phi(x) + x Phi(-x) = x
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(S.gelu_grad(x) - fd)) <= 1e-8


def _tiny(seed=1, dims=(5, 7, 6, 3)):
    rng = np.random.default_rng(seed)
    params = [(rng.normal(size=(dims[i + 1], dims[i])) / math.sqrt(dims[i]),
               rng.normal(size=dims[i + 1]) * 0.1) for i in range(len(dims) - 1)]
    X = rng.normal(size=(4, dims[0]))
    U = rng.normal(size=(4, dims[-1]))
    return params, X, U


def test_backward_fp32_matches_finite_differences():
    params, X, U = _tiny()

    def L(ps):
        y, _ = S.forward(ps, X, "fp32")
        return S.loss(y, U)

    y, cache = S.forward(params, X, "fp32")
    grads = S.backward(params, cache, y, U, "fp32")
    h = 1e-6
    for l, (Wl, bl) in enumerate(params):
        for arr, g in ((Wl, grads[l][0]), (bl, grads[l][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = L(params)
                arr[idx] = old - h
                lm = L(params)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_single_linear_layer_is_least_squares_gradient():
    """With no hidden layer the loss is a linear least-squares problem: its minimiser (from
    lstsq) has zero gradient, and the gradient is linear in the residual."""
    rng = np.random.default_rng(3)
    X, U = rng.normal(size=(12, 4)), rng.normal(size=(12, 2))
    Xa = np.hstack([X, np.ones((12, 1))])
    sol = np.linalg.lstsq(Xa, U, rcond=None)[0]          # (5 x 2)
    params = [(sol[:4].T.copy(), sol[4].copy())]
    y, cache = S.forward(params, X, "fp32")
    g = S.backward(params, cache, y, U, "fp32")[0]
    assert np.max(np.abs(g[0])) <= 1e-12 and np.max(np.abs(g[1])) <= 1e-12


def test_bf16_mode_rounds_and_stays_close():
    params, X, U = _tiny(seed=5, dims=(16, 32, 32, 8))
    y32, c32 = S.forward(params, X, "fp32")
    y16, c16 = S.forward(params, X, "bf16")
    for a in c16[0]:
        assert np.array_equal(S.bf16_round(a), a)      # every activation is a bf16 value
    assert 0 < np.max(np.abs(y16 - y32)) <= 2e-2 * np.max(np.abs(y32))
    g32 = S.backward(params, c32, y32, U, "fp32")
    g16 = S.backward(params, c16, y16, U, "bf16")
    for (a, b), (c, d) in zip(g16, g32):
        assert np.max(np.abs(a - c)) <= 3e-2 * np.max(np.abs(c))
        assert np.max(np.abs(b - d)) <= 3e-2 * np.max(np.abs(d))


def test_adamw_closed_forms():
    rng = np.random.default_rng(4)
    w0, g = rng.normal(size=50), rng.normal(size=50)
    lr, wd, eps = 1e-3, 0.01, 1e-8
    w, m, v = S.adamw_step(w0, np.zeros(50), np.zeros(50), g, 1, lr, wd=wd, eps=eps)
    # first step: bias-corrected moments are g and g^2
    assert np.allclose(w, w0 - lr * (g / (np.abs(g) + eps) + wd * w0), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 for every t (wd = 0)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        w, m, v = S.adamw_step(w, m, v, g, t, lr, eps=eps)
    assert np.allclose(w, w0 - 7 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


def test_lower_bound_is_the_riccati_value():
    for k in range(3):
        p = W.heat1d(12, 3, 6, seed=(9, k))
        red = oracle.reduce_problem(p)
        _, fstar = riccati(p)
        assert abs(S.lower_bound(red) - fstar) <= 1e-10 * abs(fstar)


def test_judge_accepts_the_optimum_and_rejects_infeasible():
    p = W.heat1d(20, 4, 8, seed=(9, 7))
    red = oracle.reduce_problem(p)
    res = oracle.solve(p, red=red)
    acc, vio, f, lb, gap = S.judge(p, res.v, red)
    assert lb <= f + 1e-12 and vio <= 1e-7
    u_free, fstar = riccati(p)
    if S.violation(p, u_free) == 0.0:      # no bound active: the IPM optimum is certified
        assert acc and gap <= 1e-6
    bad = res.v.copy()
    bad[0] = p.uu[0] + 0.5                 # control bound broken by 0.5
    acc2, vio2, *_ = S.judge(p, bad, red)
    assert not acc2 and abs(vio2 - 0.5) <= 1e-12 or vio2 > 0.5


def test_violation_scalar_closed_form():
    """ns = nu = N = 1: x1 = a x0 + b u, so the violation is max(0, x1 - xu, xl - x1,
    u - uu, ul - u)."""
    a, b, x0 = 0.8, 0.5, 0.3
    p = W.LQProblem(A=np.array([[a]]), B=np.array([[b]]), Q=np.eye(1), R=np.eye(1),
                    Qf=np.eye(1), xl=np.array([-0.5]), xu=np.array([0.4]),
                    ul=np.array([-1.0]), uu=np.array([1.0]), x0=np.array([x0]), N=1)
    for u in (-2.0, -1.0, 0.0, 0.2, 0.5, 1.5):
        x1 = a * x0 + b * u
        ref = max(0.0, x1 - 0.4, -0.5 - x1, u - 1.0, -1.0 - u)
        assert abs(S.violation(p, np.array([u])) - ref) <= 1e-15


def test_widths_and_parameter_count():
    w = S.widths(1000, 500)
    assert w == [1000, 1024, 1024, 1024, 1024, 500]
    # 1000*1024 + 1024 + 3 (1024*1024 + 1024) + 1024*500 + 500
    assert S.param_count(w) == 4_686_324
