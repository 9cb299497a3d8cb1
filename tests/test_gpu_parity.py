"""Parity of the HIP path (through the C ABI) with the CPU oracle, step by step.

Tolerances (FP64 path): the reduction, the condensed matrix and the factorisation are
compared element-wise at 1e-12 relative to the largest magnitude of the compared array
(sums of up to ~5e4 products of O(1) numbers in a different order: ~1e-14 expected);
Newton directions at 1e-9 relative (the solve amplifies rounding by cond(K), which the
test points keep below ~1e6); converged solves by the objective within 1e-8 relative and
the KKT residuals within 1e-8, with the same iteration count.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W
from test_oracle_pins import random_stable

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def cases():
    small = W.heat1d_config("small")
    ragged = W.heat1d(37, 3, 23, seed=(9, 1))                      # n = 69: two tiles, ragged
    tight = W.heat1d(60, 4, 20, seed=(0, 1), xu=0.05, x0_range=(-0.4, 0.04))
    genq = random_stable(7, 3, 9, 5)                               # dense Q, Q_f
    inf = W.heat1d(30, 2, 12, seed=(4, 4))
    inf.xu[3] = np.inf
    inf.xl[5] = -np.inf
    inf.uu[1] = np.inf
    wide = W.heat1d(50, 7, 21, seed=(8, 2))                       # n = 147: 3 tile rows
    tall = W.heat1d(130, 17, 6, seed=(5, 3))                       # ns > 64, ragged: 3 row groups
    cube = W.heat3d(3, 8)                                          # the paper's 3-D cube, m = 3
    return {"small": small, "ragged": ragged, "tight": tight, "genq": genq, "inf": inf,
            "wide": wide, "tall": tall, "cube": cube}


CASES = cases()


def rel_err(a, b):
    scale = max(1.0, float(np.max(np.abs(b))))
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / scale


@pytest.fixture(scope="module")
def problems(lib):
    out = {}
    for name, p in CASES.items():
        print(f"[parity] building {name}: ns={p.ns} nu={p.nu} N={p.N}", flush=True)
        gp = condmpc.Problem(p)
        gp.set_x0(p.x0)
        out[name] = (p, gp, oracle.reduce_problem(p))
    yield out
    for _, gp, _ in out.values():
        gp.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_reduction(problems, name):
    """Gamma, c, H, h, h0, d of Section 2 against the oracle."""
    p, gp, red = problems[name]
    ex = gp.export_dense()
    assert rel_err(ex["Gamma"], red.Gamma) <= 1e-13
    assert rel_err(ex["c"], red.c) <= 1e-13
    assert rel_err(ex["H"], red.H) <= 1e-12
    assert np.array_equal(ex["H"], ex["H"].T)
    assert rel_err(ex["h"], red.h) <= 1e-12
    assert abs(ex["h0"] - red.h0) <= 1e-12 * max(1.0, abs(red.h0))
    keep = np.isfinite(ex["d"])
    assert keep.sum() == red.d.size
    assert rel_err(ex["d"][keep], red.d) <= 1e-13


def _sigma_full(gp, red, sig_kept):
    d = gp.export_dense(gamma=False)["d"]
    keep = np.isfinite(d)
    full = np.zeros(gp.m)
    full[keep] = sig_kept
    return full, keep


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("scale", [1e-6, 1.0, 1e6])
def test_condensed_matrix(problems, name, scale):
    """K = H + J' Sigma J (eqn. (cond_KKT) left-hand side), lower triangle."""
    p, gp, red = problems[name]
    rng = np.random.default_rng(3)
    sig = scale * rng.uniform(0.01, 10.0, red.d.size)
    full, _ = _sigma_full(gp, red, sig)
    K = torch.zeros(gp.n, gp.n, dtype=torch.float64, device=DEV)
    gp.form_condensed(gpu(full), K)
    K_ref = oracle.condensed_matrix(red, sig)
    Kg = K.cpu().numpy()
    lo = np.tril_indices(gp.n)
    assert rel_err(Kg[lo], K_ref[lo]) <= 1e-12


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 127, 128, 129, 130, 257, 500])
def test_cholesky_and_solve(lib, n):
    rng = np.random.default_rng(n)
    M = rng.normal(size=(n, n))
    A = M @ M.T + n * np.eye(n)
    Kt = gpu(np.triu(np.full((n, n), 7.0), 1) + np.tril(A))     # junk above the diagonal
    info = condmpc.potrf(Kt)
    assert info == 0
    L = np.tril(Kt.cpu().numpy())
    L_ref = np.linalg.cholesky(A)
    assert rel_err(L, L_ref) <= 1e-12
    assert np.all(np.triu(Kt.cpu().numpy(), 1) == np.triu(np.full((n, n), 7.0), 1))
    b = rng.normal(size=n)
    bt = gpu(b)
    condmpc.potrs(Kt, bt)
    x_ref = np.linalg.solve(A, b)
    assert rel_err(bt.cpu().numpy(), x_ref) <= 1e-11


def test_cholesky_reports_indefinite(lib):
    n = 100
    A = np.eye(n)
    A[70, 70] = -1.0
    with pytest.raises(condmpc.CmpcError) as e:
        condmpc.potrf(gpu(A))
    assert e.value.code == condmpc.ERR_CHOLESKY
    assert "71" in str(e.value)


@pytest.mark.parametrize("name", sorted(CASES))
def test_newton_step(problems, name):
    """One condensed Newton direction and its step lengths from a random interior point."""
    p, gp, red = problems[name]
    rng = np.random.default_rng(11)
    mk = red.d.size
    v = rng.uniform(-0.2, 0.2, gp.n)
    s = rng.uniform(0.05, 1.0, mk)
    lam = rng.uniform(0.01, 2.0, mk)
    z = rng.uniform(0.01, 2.0, mk)
    mu, tau = 0.03, 0.99
    ref = oracle.condensed_step(red, v, s, lam, z, mu)
    d = gp.export_dense(gamma=False)["d"]
    keep = np.isfinite(d)

    def full(x, fill):
        f = np.full(gp.m, fill)
        f[keep] = x
        return gpu(f)
    out = gp.newton_step(gpu(v), full(s, 1.0), full(lam, 0.0), full(z, 0.0), mu, tau)
    assert rel_err(out["pv"].cpu().numpy(), ref["pv"]) <= 1e-9
    for k in ("ps", "plam", "pz"):
        g = out[k].cpu().numpy()
        assert rel_err(g[keep], ref[k]) <= 1e-9, k
        assert np.all(g[~keep] == 0.0)
    a_ref = oracle.fraction_to_boundary(s, ref["ps"], tau)
    az_ref = oracle.fraction_to_boundary(z, ref["pz"], tau)
    assert out["alpha"] == pytest.approx(a_ref, rel=1e-9)
    assert out["alpha_z"] == pytest.approx(az_ref, rel=1e-9)


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_solve(problems, name):
    """Algorithm 1 end to end against the oracle: same status and iteration count,
    objective within 1e-8 relative, KKT residuals within 1e-8."""
    p, gp, red = problems[name]
    ref = oracle.solve(p, red=red)
    res = gp.solve()
    print(f"[parity] {name}: gpu iters {res['iters']} obj {res['obj']:.12e} | "
          f"oracle iters {ref.iters} obj {ref.obj:.12e}", flush=True)
    assert res["status"] == condmpc.OK == ref.status
    assert res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
    assert res["compl_res"] <= 1e-8
    u, x = gp.solution()
    assert rel_err(u, ref.v) <= 1e-6
    assert rel_err(x, ref.x) <= 1e-6
    # the states returned are the simulated ones of the returned controls
    assert rel_err(x, oracle.simulate(p, u)) <= 1e-12
    # weak duality: objective within the final duality gap of the oracle's
    assert abs(res["gap"] - ref.gap) <= 1e-6 * max(ref.gap, 1e-12) + 1e-12


@pytest.mark.parametrize("dims", [(40, 8, 40), (30, 10, 60), (20, 13, 50)])
def test_full_solve_many_tiles(lib, dims):
    """Solves whose K spans 5, 10 and 11 (ragged) 64-row tiles: the factorisation's fused
    forward substitution (blocks up to nt-3 inside the Cholesky launches) followed by the
    unrolled (nt <= 8) and the looped (nt > 8) one-workgroup solve, against the oracle."""
    ns, nu, N = dims
    p = W.heat1d(ns, nu, N, seed=(17, ns))
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    ref = oracle.solve(p)
    res = gp.solve()
    u, x = gp.solution()
    gp.close()
    print(f"[parity] n={nu * N}: gpu iters {res['iters']} obj {res['obj']:.12e} | "
          f"oracle iters {ref.iters} obj {ref.obj:.12e}", flush=True)
    assert res["status"] == condmpc.OK == ref.status
    assert res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8 and res["compl_res"] <= 1e-8
    assert rel_err(u, ref.v) <= 1e-6


def test_repeat_solve_is_deterministic(problems):
    p, gp, red = problems["wide"]
    r1 = gp.solve()
    u1, _ = gp.solution(with_x=False)
    r2 = gp.solve()
    u2, _ = gp.solution(with_x=False)
    assert r1["iters"] == r2["iters"] and r1["obj"] == r2["obj"]
    assert np.array_equal(u1, u2)


def test_new_x0_reuses_problem(problems):
    p, gp, red = problems["small"]
    x0b = np.random.default_rng(77).uniform(-0.3, 0.3, p.ns)
    pb = p.with_x0(x0b)
    gp.set_x0(x0b)
    res = gp.solve()
    ref = oracle.solve(pb)
    gp.set_x0(p.x0)
    assert res["status"] == 0 and res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))


def test_x0_outside_bounds_rejected(problems):
    p, gp, red = problems["small"]
    bad = p.x0.copy()
    bad[3] = 0.9
    with pytest.raises(condmpc.CmpcError) as e:
        gp.set_x0(bad)
    assert e.value.code == condmpc.ERR_X0_BOUNDS
    bad[3] = np.nan
    with pytest.raises(condmpc.CmpcError) as e:
        gp.set_x0(bad)
    assert e.value.code == condmpc.ERR_NONFINITE
    gp.set_x0(p.x0)


def test_iteration_limit(problems):
    p, gp, red = problems["tight"]
    res = gp.solve(max_iter=2)
    assert res["status"] == condmpc.MAX_ITER and res["iters"] == 2
    ref = oracle.solve(p, red=red, max_iter=2)
    assert ref.status == oracle.STATUS_MAX_ITER
    assert abs(res["obj"] - ref.obj) <= 1e-9 * max(1.0, abs(ref.obj))


def test_device_x0_checked_on_device(problems):
    """A device-resident x0 is validated on the GPU; the next solve reports the error."""
    p, gp, red = problems["small"]
    bad = p.x0.copy()
    bad[7] = 0.75
    gp.set_x0(gpu(bad))
    with pytest.raises(condmpc.CmpcError) as e:
        gp.solve()
    assert e.value.code == condmpc.ERR_X0_BOUNDS
    bad[7] = np.inf
    gp.set_x0(gpu(bad))
    with pytest.raises(condmpc.CmpcError) as e:
        gp.solve()
    assert e.value.code == condmpc.ERR_NONFINITE
    gp.set_x0(gpu(p.x0))
    res = gp.solve()
    ref = oracle.solve(p, red=red)
    assert res["status"] == 0 and res["iters"] == ref.iters


@pytest.mark.parametrize("n", [1000, 1111, 4097])
def test_cholesky_large(lib, n):
    rng = np.random.default_rng(n)
    M = rng.normal(size=(n, n)) / np.sqrt(n)
    A = M @ M.T + np.diag(rng.uniform(0.5, 2.0, n))
    Kt = gpu(np.tril(A))
    condmpc.potrf(Kt)
    L = np.tril(Kt.cpu().numpy())
    assert rel_err(L, np.linalg.cholesky(A)) <= 1e-11
    b = rng.normal(size=n)
    bt = gpu(b)
    condmpc.potrs(Kt, bt)          # n <= 4096: one workgroup; larger: block steps
    assert rel_err(bt.cpu().numpy(), np.linalg.solve(A, b)) <= 1e-10


# ----------------------------------------------------------------- mixed precision (FP32 SYRK)

@pytest.mark.parametrize("name", ["small", "ragged", "wide", "tight"])
def test_condensed_matrix_fp32(problems, name):
    """The FP32-MFMA SYRK (FP64 H and diagonal) against the FP64 oracle: products rounded to
    FP32 (u = 6e-8) summed over <= 1e4 terms in blocks -> within 1e-5 of the largest entry."""
    p, gp, red = problems[name]
    rng = np.random.default_rng(5)
    sig = rng.uniform(0.01, 10.0, red.d.size)
    full, _ = _sigma_full(gp, red, sig)
    K = torch.zeros(gp.n, gp.n, dtype=torch.float64, device=DEV)
    gp.form_condensed(gpu(full), K, precision=condmpc.FP32_SYRK)
    K_ref = oracle.condensed_matrix(red, sig)
    lo = np.tril_indices(gp.n)
    err = rel_err(K.cpu().numpy()[lo], K_ref[lo])
    assert 0 < err <= 1e-5   # nonzero: the low-precision kernel really ran


@pytest.mark.parametrize("name", ["small", "ragged", "wide", "tight", "inf", "genq"])
def test_mixed_precision_solve(problems, name):
    """FP32 SYRK + FP64 Cholesky + FP64 iterative refinement meets the FP64 bar: objective
    within 1e-8 relative of the oracle, KKT residuals within 1e-8."""
    p, gp, red = problems[name]
    ref = oracle.solve(p, red=red)
    res = gp.solve(precision=condmpc.FP32_SYRK)
    print(f"[mixed] {name}: iters {res['iters']} (oracle {ref.iters}) switch "
          f"{res['precision_switch_iter']} refine {res['refine_steps']} obj rel "
          f"{abs(res['obj'] - ref.obj) / max(1, abs(ref.obj)):.2e}", flush=True)
    assert res["status"] == condmpc.OK
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8 and res["compl_res"] <= 1e-8
    assert abs(res["iters"] - ref.iters) <= 2
    u, _ = gp.solution(with_x=False)
    assert rel_err(u, ref.v) <= 1e-6


@pytest.mark.parametrize("name", ["small", "ragged", "wide"])
def test_condensed_matrix_bf16(problems, name):
    """The BF16-MFMA SYRK (Gamma rounded to bfloat16, D-scaled operand rounded again, float32
    accumulation; FP64 H and diagonal): each product carries <= 3 roundings of 2^-8, so the
    error is within 2e-2 of the largest entry, and nonzero."""
    p, gp, red = problems[name]
    rng = np.random.default_rng(6)
    sig = rng.uniform(0.01, 10.0, red.d.size)
    full, _ = _sigma_full(gp, red, sig)
    K = torch.zeros(gp.n, gp.n, dtype=torch.float64, device=DEV)
    gp.form_condensed(gpu(full), K, precision=condmpc.BF16_SYRK)
    K_ref = oracle.condensed_matrix(red, sig)
    lo = np.tril_indices(gp.n)
    err = rel_err(K.cpu().numpy()[lo], K_ref[lo])
    print(f"[bf16] {name}: K rel err {err:.2e}", flush=True)
    assert 0 < err <= 2e-2


@pytest.mark.parametrize("name", ["small", "ragged", "wide", "tight", "inf", "genq"])
def test_bf16_mixed_solve(problems, name):
    """BF16 start, staged FP32 -> FP64, equilibrated FP64 Cholesky and FP64 refinement: the
    FP64 bar on the objective and the KKT residuals."""
    p, gp, red = problems[name]
    ref = oracle.solve(p, red=red)
    res = gp.solve(precision=condmpc.BF16_SYRK)
    print(f"[bf16 mixed] {name}: iters {res['iters']} (oracle {ref.iters}) switch "
          f"{res['precision_switch_iter']} refine {res['refine_steps']} obj rel "
          f"{abs(res['obj'] - ref.obj) / max(1, abs(ref.obj)):.2e}", flush=True)
    assert res["status"] == condmpc.OK
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8 and res["compl_res"] <= 1e-8
    assert abs(res["iters"] - ref.iters) <= 4
    u, _ = gp.solution(with_x=False)
    assert rel_err(u, ref.v) <= 1e-6


@pytest.mark.parametrize("name", ["small", "tight", "wide"])
def test_equilibrated_fp64_solve(problems, name):
    """Factoring S K S (S = diag(K)^-1/2) instead of K changes only rounding: same status and
    iteration count as the oracle, objective within 1e-8."""
    p, gp, red = problems[name]
    ref = oracle.solve(p, red=red)
    res = gp.solve(equilibrate=1)
    assert res["status"] == condmpc.OK and res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8


# ----------------------------------------------------------------- the benchmarked workload
CONFIG2 = [("seed0", 0, {}), ("seed1", 1, {}), ("seed2", 2, {}),
           ("tight", 0, {"xu": 0.05, "x0_range": (-0.4, 0.04)})]


@pytest.fixture(scope="module")
def config2(lib):
    """The benchmarked 1-D heat workload (ns 1000, nu 10, N 50: K 500 x 500, 50,000 state
    rows) for three x0 seeds and the tight-bound variant (thousands of active rows)."""
    out = {}
    for name, inst, kw in CONFIG2:
        p = W.heat1d_config("1d", instance=inst, **kw)
        print(f"[config2] oracle {name}", flush=True)
        out[name] = (p, oracle.solve(p))
    yield out


@pytest.mark.parametrize("name", [c[0] for c in CONFIG2])
def test_config2_matches_oracle(config2, name):
    """FP64: same status and iteration count as the oracle, objective within 1e-8, residuals
    within 1e-8; FP32 and BF16 starts: the same bar on the objective and the residuals."""
    p, ref = config2[name]
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    try:
        for prec, label in ((condmpc.FP64, "fp64"), (condmpc.FP32_SYRK, "fp32"),
                            (condmpc.BF16_SYRK, "bf16")):
            res = gp.solve(precision=prec)
            u, x = gp.solution()
            err = abs(res["obj"] - ref.obj) / max(1.0, abs(ref.obj))
            print(f"[config2] {name} {label}: iters {res['iters']} (oracle {ref.iters}) obj "
                  f"rel err {err:.2e} |u-u*| {rel_err(u, ref.v):.2e} switch "
                  f"{res['precision_switch_iter']} refine {res['refine_steps']}", flush=True)
            assert res["status"] == condmpc.OK == ref.status
            if prec == condmpc.FP64:
                assert res["iters"] == ref.iters
            else:
                assert abs(res["iters"] - ref.iters) <= 4
            assert err <= 1e-8
            assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
            assert res["compl_res"] <= 1e-8
            assert rel_err(u, ref.v) <= 1e-6 and rel_err(x, ref.x) <= 1e-6
    finally:
        gp.close()


def test_config2_log_follows_the_oracle_barrier_sequence(config2):
    """The per-iteration log of an FP64 solve: one line per iteration and a final one; its
    barrier parameters are the oracle's, iteration by iteration."""
    p, ref = config2["seed0"]
    rec = oracle.solve(p, record=True)
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    lines = []
    res = gp.solve(log=lines.append)
    gp.close()
    print("\n".join(lines), flush=True)
    assert len(lines) == res["iters"] + 1
    assert lines[-1].startswith(f"stop after {res['iters']} iterations")
    mus = [float(l.split(" mu ")[1].split()[0]) for l in lines[:-1]]
    np.testing.assert_allclose(mus, [h["mu"] for h in rec.history], rtol=1e-3)


# ----------------------------------------------------------------- precision-level moves
@pytest.mark.parametrize("start", [condmpc.FP32_SYRK, condmpc.BF16_SYRK])
def test_precision_moves_by_refinement(problems, start):
    """refine_contract = 0 counts every refinement step of an iteration after its first as not
    contracting, and mu_switch = 0 disables the switch by the barrier parameter, so the only
    way up is refinement: the SYRK moves up one level per two counts (BF16 -> FP32 -> FP64,
    or FP32 -> FP64).  An iteration whose first step already reaches 1e-12 counts nothing,
    so the move comes once K is ill-conditioned enough to need two steps; it must come
    before convergence, and the solve still meets the FP64 bar."""
    p, gp, red = problems["tight"]
    ref = oracle.solve(p, red=red)
    res = gp.solve(precision=start, refine_contract=0.0, mu_switch=0.0)
    print(f"[moves] start {start}: switch {res['precision_switch_iter']} refine "
          f"{res['refine_steps']} iters {res['iters']}", flush=True)
    assert res["status"] == condmpc.OK
    assert 1 <= res["precision_switch_iter"] < res["iters"]
    assert res["refine_steps"] >= (4 if start == condmpc.BF16_SYRK else 2)
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8


def test_precision_switch_by_barrier(problems):
    """Default rule, FP32 start: refinement runs (steps > 0) and the SYRK moves to FP64 no
    later than the first iteration whose barrier parameter is below mu_switch = 1e-6."""
    p, gp, red = problems["tight"]
    rec = oracle.solve(p, red=red, record=True)
    res = gp.solve(precision=condmpc.FP32_SYRK)
    first_small = next(h["k"] for h in rec.history if h["mu"] < 1e-6)
    print(f"[switch] FP32 start: switch {res['precision_switch_iter']} (oracle mu < 1e-6 at "
          f"{first_small}) refine {res['refine_steps']}", flush=True)
    assert res["refine_steps"] > 0
    assert 0 < res["precision_switch_iter"] <= first_small + 2


def test_no_refinement_no_moves(problems):
    """max_refine = 0 and mu_switch = 0: no refinement step and no level change (the FP32
    Newton directions are used as they are) over the first iterations."""
    p, gp, red = problems["small"]
    res = gp.solve(precision=condmpc.FP32_SYRK, max_refine=0, mu_switch=0.0, max_iter=6)
    assert res["refine_steps"] == 0 and res["precision_switch_iter"] == -1
    assert res["status"] in (condmpc.OK, condmpc.MAX_ITER)


# ----------------------------------------------------------------- the 2-D 70 x 70 workload
def test_heat2d_70x70_reduced_horizon(lib):
    """The 2-D heat grid of the largest workload (70 x 70 interior nodes, 4900 states, 20
    boundary actuators) at horizon N = 12 (K 240 x 240, 58,800 state rows) against the
    oracle: FP64 with the oracle's iteration count, FP32 and BF16 starts on the FP64 bar."""
    p = W.heat2d(70, 5, 12, seed=(2, 0))
    ref = oracle.solve(p)
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    try:
        for prec in (condmpc.FP64, condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            res = gp.solve(precision=prec)
            u, _ = gp.solution(with_x=False)
            print(f"[heat2d] prec {prec}: iters {res['iters']} (oracle {ref.iters}) obj "
                  f"{res['obj']:.12e} vs {ref.obj:.12e}", flush=True)
            assert res["status"] == condmpc.OK == ref.status
            if prec == condmpc.FP64:
                assert res["iters"] == ref.iters
            assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
            assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
            assert rel_err(u, ref.v) <= 1e-6
    finally:
        gp.close()


def test_heat2d_70x70_full_size(lib):
    """The largest workload at its full size (70 x 70 grid, N = 100: K 2000 x 2000, 490,000
    state rows), in the configuration the benchmark times.  The oracle's dense reduction does
    not fit here, so every result is checked through properties that hold at any size and
    that the oracle computes on the CPU one by one: the objective of the returned controls by
    forward simulation (eqn. (dyn)) equals the reported one, the simulated states and the
    controls keep their bounds, the FP64 KKT residuals meet the bar, and the FP32- and
    BF16-start solves reach the FP64 solve's objective within 1e-8."""
    p = W.heat2d(**W.CONFIG_2D, seed=(2, 0))
    print(f"[heat2d full] ns {p.ns} nu {p.nu} N {p.N}", flush=True)
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    objs = {}
    try:
        for prec in (condmpc.FP64, condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            res = gp.solve(precision=prec)
            u, _ = gp.solution(with_x=False)
            f_sim = oracle.sparse_objective(p, u)
            x = oracle.simulate(p, u)
            viol = max(float(np.max(x - np.tile(p.xu, p.N))),
                       float(np.max(np.tile(p.xl, p.N) - x)),
                       float(np.max(u - np.tile(p.uu, p.N))),
                       float(np.max(np.tile(p.ul, p.N) - u)))
            print(f"[heat2d full] prec {prec}: status {res['status']} iters {res['iters']} obj "
                  f"{res['obj']:.12e} simulated {f_sim:.12e} violation {viol:.2e} switch "
                  f"{res['precision_switch_iter']} refine {res['refine_steps']}", flush=True)
            assert res["status"] == condmpc.OK
            assert abs(res["obj"] - f_sim) <= 1e-10 * max(1.0, abs(f_sim))
            assert viol <= 1e-9
            assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
            objs[prec] = res["obj"]
    finally:
        gp.close()
    f64 = objs[condmpc.FP64]
    for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
        assert abs(objs[prec] - f64) <= 1e-8 * max(1.0, abs(f64))


def test_cube_m13_T250_full_size(lib):
    """The paper's largest 3-D cube shape (m = 13 nodes per dimension, T = 250: ns = 2197,
    K 1500 x 1500, 549,250 state rows; Table 2's shape), in the configuration the benchmark's
    paper-shapes leg times.  Too large for the oracle's dense reduction, so checked through
    properties the oracle computes one by one on the CPU: the objective of the returned
    controls by forward simulation equals the reported one, states and controls keep their
    bounds, the FP64 KKT residuals meet the bar, and the FP32- and BF16-start solves reach the
    FP64 objective within 1e-8."""
    p = W.heat3d(13, 250)
    print(f"[cube full] ns {p.ns} nu {p.nu} N {p.N}", flush=True)
    gp = condmpc.Problem(p)
    gp.set_x0(p.x0)
    objs = {}
    try:
        for prec in (condmpc.FP64, condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            res = gp.solve(precision=prec)
            u, _ = gp.solution(with_x=False)
            f_sim = oracle.sparse_objective(p, u)
            x = oracle.simulate(p, u)
            viol = max(float(np.max(x - np.tile(p.xu, p.N))),
                       float(np.max(np.tile(p.xl, p.N) - x)),
                       float(np.max(u - np.tile(p.uu, p.N))),
                       float(np.max(np.tile(p.ul, p.N) - u)))
            print(f"[cube full] prec {prec}: status {res['status']} iters {res['iters']} obj "
                  f"{res['obj']:.12e} simulated {f_sim:.12e} violation {viol:.2e} switch "
                  f"{res['precision_switch_iter']} refine {res['refine_steps']}", flush=True)
            assert res["status"] == condmpc.OK
            assert abs(res["obj"] - f_sim) <= 1e-10 * max(1.0, abs(f_sim))
            assert viol <= 1e-9
            assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8
            objs[prec] = res["obj"]
    finally:
        gp.close()
    f64 = objs[condmpc.FP64]
    for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
        assert abs(objs[prec] - f64) <= 1e-8 * max(1.0, abs(f64))
