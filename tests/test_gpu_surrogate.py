"""The surrogate policy on the GPU against the CPU oracle (oracle/surrogate.py).

* forward outputs and gradients of every tensor: FP32 test mode within 1e-5 relative per
  tensor, BF16 mode within 2e-2 (same rounding points as the oracle);
* AdamW trajectory over several steps against the oracle's updates;
* the FP64 judge (violation, objective, lower bound, decision) against the oracle's;
* end to end: the IPM generates the training data, the network trains on the GPU, and
  every answer of cmpc_surrogate_solve is either certified (and the oracle's judge agrees)
  or is the IPM's own solution; the network answers a share of the queries without a solve.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import surrogate as S
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu

NS, NU, N = 40, 4, 8          # n = 32 controls
HIDDEN, DEPTH = 64, 2


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def tensor_rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.fixture(scope="module")
def setup(lib):
    prob = W.heat1d(NS, NU, N, seed=(21, 0))
    gp = condmpc.Problem(prob)
    gp.set_x0(prob.x0)
    widths = W.mlp_widths(NS, NU * N, HIDDEN, DEPTH)
    init = W.mlp_init(widths, seed=7)
    yield prob, gp, widths, init
    gp.close()


def unpack_grads(flat, widths):
    return W.unpack_params(flat, widths)


@pytest.mark.parametrize("mode,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_forward_and_gradients_match_oracle(setup, mode, tol):
    prob, gp, widths, init = setup
    prec = condmpc.MLP_FP32 if mode == "fp32" else condmpc.MLP_BF16
    net = condmpc.Mlp(gp, init, HIDDEN, DEPTH, prec)
    count = 100                                     # not a multiple of 64: padded rows
    X = W.smooth_x0(NS, count, seed=31)
    U = np.random.default_rng(32).uniform(-1, 1, size=(count, NU * N))
    g, loss, y = net.gradients(gpu(X), gpu(U))
    params = W.unpack_params(init, widths)
    yo, cache = S.forward(params, X, mode)
    go = S.backward(params, cache, yo, U, mode)
    print(f"[surrogate] {mode}: y rel {tensor_rel(y, yo):.2e} loss {loss:.6e} vs "
          f"{S.loss(yo, U):.6e}", flush=True)
    assert tensor_rel(y, yo) <= tol
    assert abs(loss - S.loss(yo, U)) <= tol * S.loss(yo, U)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(unpack_grads(g, widths), go)):
        eW, eb = tensor_rel(gW, oW), tensor_rel(gb, ob)
        print(f"[surrogate] {mode} layer {l + 1}: dW rel {eW:.2e} db rel {eb:.2e}", flush=True)
        assert eW <= tol and eb <= tol
    net.close()


def test_adamw_trajectory_matches_oracle(setup):
    prob, gp, widths, init = setup
    net = condmpc.Mlp(gp, init, HIDDEN, DEPTH, condmpc.MLP_FP32)
    count, steps, lr, wd = 64, 3, 1e-3, 1e-2
    X = W.smooth_x0(NS, count, seed=41)
    U = np.random.default_rng(42).uniform(-1, 1, size=(count, NU * N))
    net.train(gpu(X), gpu(U), batch=count, epochs=steps, lr=lr, lr_final=lr, weight_decay=wd)
    got = W.unpack_params(net.params(), widths)
    params = [(Wl.copy(), bl.copy()) for Wl, bl in W.unpack_params(init, widths)]
    mom = [[np.zeros_like(Wl), np.zeros_like(Wl), np.zeros_like(bl), np.zeros_like(bl)]
           for Wl, bl in params]
    small = [np.zeros_like(Wl, dtype=bool) for Wl, _ in params]
    for t in range(1, steps + 1):
        y, cache = S.forward(params, X, "fp32")
        grads = S.backward(params, cache, y, U, "fp32")
        for l, ((Wl, bl), (gW, gb)) in enumerate(zip(params, grads)):
            small[l] |= np.abs(gW) < 1e-7
            m = mom[l]
            Wn, m[0], m[1] = S.adamw_step(Wl, m[0], m[1], gW, t, lr, wd=wd)
            bn, m[2], m[3] = S.adamw_step(bl, m[2], m[3], gb, t, lr, wd=0.0)
            params[l] = (Wn, bn)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(got, params)):
        dW = np.abs(gW - oW)[~small[l]]
        assert np.max(dW) <= 2e-3 * lr * steps, f"layer {l + 1}: {np.max(dW)}"
        assert np.max(np.abs(gb - ob)) <= 2e-3 * lr * steps
    net.close()


def test_judge_matches_oracle(setup):
    prob, gp, widths, init = setup
    net = condmpc.Mlp(gp, init, HIDDEN, DEPTH, condmpc.MLP_BF16)
    count = 24
    X = W.smooth_x0(NS, count, seed=51)
    red = None
    answers = []
    for k in range(count):
        pk = prob.with_x0(X[k])
        if k % 3 == 0:
            u = oracle.solve(pk).v
        elif k % 3 == 1:
            u = np.clip(oracle.solve(pk).v + np.random.default_rng(k).normal(0, 0.05, NU * N),
                        -1, 1)
        else:
            u = np.zeros(NU * N)
        answers.append(u)
    Uq = np.array(answers)
    acc, vio, f, lb = net.judge(gpu(X), gpu(Uq))
    for k in range(count):
        pk = prob.with_x0(X[k])
        red = oracle.reduce_problem(pk)
        a, v, fo, lbo, gap = S.judge(pk, Uq[k], red)
        assert abs(vio[k] - v) <= 1e-12 + 1e-10 * abs(v)
        assert abs(f[k] - fo) <= 1e-10 * abs(fo)
        assert abs(lb[k] - lbo) <= 1e-9 * abs(lbo)
        near = abs(v - S.VIOLATION_TOL) < 1e-9 or abs(gap - S.GAP_TOL) < 1e-6
        if not near:
            assert bool(acc[k]) == a, f"query {k}: gpu {acc[k]} oracle {a} (vio {v}, gap {gap})"
    assert acc.any() and not acc.all()
    net.close()


def ipm_solutions(gp, X):
    """Solutions of Algorithm 1 on the GPU for each row of X (device tensors)."""
    Xd = gpu(X)
    U = torch.empty((X.shape[0], gp.n), dtype=torch.float64, device="cuda:0")
    for k in range(X.shape[0]):
        gp.set_x0(Xd[k])
        r = gp.solve()
        assert r["status"] == condmpc.OK
        u, _ = gp.solution(with_x=False)
        U[k] = torch.from_numpy(u)
    return Xd, U


def test_surrogate_end_to_end(lib):
    """IPM-generated data, GPU training, then answers that are either certified by the judge
    (the oracle's judge agrees) or are the IPM's own solution.  The certificate compares with
    the unconstrained minimum, so even the exact optimum is certified only where no bound is
    active at it; the network must reach at least half of that ceiling."""
    prob = W.heat1d(NS, NU, N, seed=(21, 1), ub=3.0)
    gp = condmpc.Problem(prob)
    gp.set_x0(prob.x0)
    hidden, depth = 256, 4
    widths = W.mlp_widths(NS, NU * N, hidden, depth)
    ntrain, nquery, epochs = 4096, 256, 300
    Xtr = W.smooth_x0(NS, ntrain, seed=61)
    t0 = time.perf_counter()
    Xd, Ud = ipm_solutions(gp, Xtr)
    t_data = time.perf_counter() - t0
    net = condmpc.Mlp(gp, W.mlp_init(widths, seed=7), hidden, depth, condmpc.MLP_BF16)
    order = W.shuffle_order(ntrain, epochs, seed=62)
    losses = net.train(Xd, Ud, order=order, batch=256, epochs=epochs, lr=1e-3, lr_final=1e-6)
    print(f"[surrogate] data {t_data:.2f} s; loss {losses[0]:.3e} -> {losses[-1]:.3e}",
          flush=True)
    assert losses[-1] < 0.01 * losses[0]
    Xq = W.smooth_x0(NS, nquery, seed=63)
    Xqd, Uqd = ipm_solutions(gp, Xq)
    ceiling, *_ = net.judge(Xqd, Uqd)             # the exact optima, judged the same way
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, acc, rep = net.solve(Xqd)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    ua = u.cpu().numpy()
    t0 = time.perf_counter()
    ipm_solutions(gp, Xq[:64])
    t_ipm = (time.perf_counter() - t0) / 64 * nquery
    print(f"[surrogate] accepted {rep['accepted']}/{nquery} (exact optima: {int(ceiling.sum())})"
          f", fallback {rep['fallback_solved']} (failed {rep['fallback_failed']}), max gap "
          f"{rep['max_gap_accepted']:.2e}; surrogate {t_sur * 1e3:.1f} ms vs IPM only "
          f"{t_ipm * 1e3:.1f} ms", flush=True)
    assert rep["count"] == nquery and rep["accepted"] == int(acc.sum())
    assert rep["accepted"] + rep["fallback_solved"] == nquery
    for k in range(nquery):
        pk = prob.with_x0(Xq[k])
        red = oracle.reduce_problem(pk)
        if acc[k]:
            a, v, f, lb, gap = S.judge(pk, ua[k], red)
            assert v <= S.VIOLATION_TOL * (1 + 1e-6) and gap <= S.GAP_TOL * (1 + 1e-6)
        elif k % 8 == 0:
            ref = oracle.solve(pk, red=red)
            assert np.max(np.abs(ua[k] - ref.v)) <= 1e-6 * max(1.0, np.max(np.abs(ref.v)))
    # what the network gains: queries answered, with a certificate, without a solve
    assert ceiling.sum() >= nquery // 4
    assert rep["accepted"] >= ceiling.sum() // 2
    # the same queries with the rejected ones solved together on a batch of copies of the
    # problem, each from the network's answer (warm start): same decisions, same optima
    fb = condmpc.Batch([prob] * 16, with_x0=False)
    net.set_fallback(fb, warm=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u2, acc2, rep2 = net.solve(Xqd)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    print(f"[surrogate] batched warm fallback: {rep2['fallback_solved']} solved in "
          f"{t_bat * 1e3:.1f} ms (one by one, cold: {t_sur * 1e3:.1f} ms)", flush=True)
    assert np.array_equal(acc2, acc) and rep2["fallback_solved"] == rep["fallback_solved"]
    u2a = u2.cpu().numpy()
    assert np.array_equal(u2a[acc], ua[acc])
    for k in np.flatnonzero(~acc)[::4]:
        pk = prob.with_x0(Xq[k])
        ref = oracle.solve(pk)
        assert np.max(np.abs(u2a[k] - ref.v)) <= 1e-6 * max(1.0, np.max(np.abs(ref.v)))
    net.set_fallback(None)
    fb.close()
    net.close()
    gp.close()
