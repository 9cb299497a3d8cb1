"""Ragged batches on the GPU (cmpc_batch_*) against the CPU oracle and against the
single-instance solve.

* every instance of a small ragged batch (uneven ns, nu, N; one tile column or several;
  ragged last tiles; an instance with infinite bounds) matches the oracle as a single solve
  does: same status and iteration count, objective within 1e-8, KKT residuals within 1e-8;
* FP64 batch iterates equal the single-instance solve of the same instance bit for bit
  (fixed-order reductions and the same block decomposition per instance);
* the FP32-SYRK batch (FP64 Cholesky and refinement) reaches the same optimum;
* the autotuner records its choice in the tuning table, later solves follow it, and the
  bitwise agreement still holds after tuning;
* error paths: missing x0, iteration limit, instance handles.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def ragged_probs():
    """Uneven instances: sizes drawn like the batch workload but small enough for the oracle,
    plus fixed edge shapes (n = 64 exactly, n = 65, a single-tile n, infinite bounds)."""
    probs = W.batch_instances(count=7, seed=11, ns_range=(20, 90), nu_range=(2, 6),
                              N_range=(4, 24))
    probs.append(W.heat1d(40, 4, 16, seed=(11, 100), name="n64"))       # n = 64: one tile
    probs.append(W.heat1d(33, 5, 13, seed=(11, 101), name="n65"))       # n = 65: ragged tile
    probs.append(W.heat1d(25, 3, 5, seed=(11, 102), name="n15"))        # tiny single tile
    inf = W.heat1d(30, 3, 9, seed=(11, 103), name="inf")
    xu = inf.xu.copy()
    xu[::3] = np.inf
    inf.xu = xu
    probs.append(inf)
    return probs


@pytest.fixture(scope="module")
def batch(lib):
    probs = ragged_probs()
    condmpc.tune_clear()
    b = condmpc.Batch(probs)
    refs = [oracle.solve(p) for p in probs]
    yield probs, b, refs
    b.close()
    condmpc.tune_clear()


def check_against_oracle(tag, res, ref, u, iters_equal=True):
    print(f"[batch] {tag}: gpu iters {res['iters']} obj {res['obj']:.12e} | "
          f"oracle iters {ref.iters} obj {ref.obj:.12e}", flush=True)
    assert res["status"] == condmpc.OK == ref.status
    if iters_equal:
        assert res["iters"] == ref.iters
    assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
    assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8 and res["compl_res"] <= 1e-8
    assert rel_err(u, ref.v) <= 1e-6


def test_batch_fp64_matches_oracle(batch):
    probs, b, refs = batch
    rc, results = b.solve()
    assert rc == condmpc.OK
    iters = set()
    for i, (p, res, ref) in enumerate(zip(probs, results, refs)):
        u, x = b[i].solution()
        check_against_oracle(f"{i} {p.name}", res, ref, u)
        assert rel_err(x, oracle.simulate(p, u)) <= 1e-12
        iters.add(res["iters"])
    # instances stop at different iterations and the finished ones are predicated off
    assert len(iters) > 1


def test_batch_fp64_bitwise_equals_single(batch):
    probs, b, refs = batch
    b.solve()
    for i in range(len(probs)):
        ub, _ = b[i].solution(with_x=False)
        vb, sb, lb, zb = b[i].iterate()
        single = condmpc.Problem(probs[i])
        single.set_x0(probs[i].x0)
        r = single.solve()
        us, _ = single.solution(with_x=False)
        vs, ss, ls, zs = single.iterate()
        single.close()
        assert np.array_equal(ub, us), f"instance {i}: u differs"
        assert np.array_equal(sb, ss) and np.array_equal(lb, ls) and np.array_equal(zb, zs)


def test_batch_fp32_syrk_reaches_the_optimum(batch):
    probs, b, refs = batch
    rc, results = b.solve(precision=condmpc.FP32_SYRK)
    assert rc == condmpc.OK
    for i, (res, ref) in enumerate(zip(results, refs)):
        u, _ = b[i].solution(with_x=False)
        check_against_oracle(f"fp32 {i}", res, ref, u, iters_equal=False)
        assert abs(res["iters"] - ref.iters) <= 3


def test_batch_repeat_is_deterministic(batch):
    probs, b, refs = batch
    b.solve()
    u1 = [b[i].solution(with_x=False)[0] for i in range(len(probs))]
    b.solve()
    u2 = [b[i].solution(with_x=False)[0] for i in range(len(probs))]
    assert all(np.array_equal(a, c) for a, c in zip(u1, u2))


def test_batch_new_x0_per_instance(batch):
    probs, b, refs = batch
    i = 2
    x0b = np.random.default_rng(5).uniform(-0.3, 0.3, probs[i].ns)
    b[i].set_x0(x0b)
    rc, results = b.solve()
    ref = oracle.solve(probs[i].with_x0(x0b))
    u, _ = b[i].solution(with_x=False)
    b[i].set_x0(probs[i].x0)
    assert rc == condmpc.OK
    check_against_oracle("new x0", results[i], ref, u)


def test_tune_records_choice_and_keeps_bitwise(batch):
    probs, b, refs = batch
    rep = b.tune(condmpc.FP64)
    print(f"[batch] tune: {rep}", flush=True)
    assert rep["candidates"] == 12
    assert rep["quantum"] in (3000, 6000, 12000, 24000, 48000, 96000)
    assert 0 < rep["syrk_us"] <= rep["default_us"] * 1.0000001
    for i in range(len(probs)):
        n, mx = b[i].n, b[i].mx
        assert condmpc.tune_lookup(n, mx, condmpc.FP64) == (rep["quantum"], rep["persistent"])
    rc, results = b.solve()
    assert rc == condmpc.OK
    for i in (0, 3, len(probs) - 1):
        ub, _ = b[i].solution(with_x=False)
        single = condmpc.Problem(probs[i])  # plans from the tuning table
        single.set_x0(probs[i].x0)
        single.solve()
        us, _ = single.solution(with_x=False)
        single.close()
        assert np.array_equal(ub, us)
        check_against_oracle(f"tuned {i}", results[i], refs[i], ub)
    condmpc.tune_clear()
    assert condmpc.tune_lookup(b[0].n, b[0].mx, condmpc.FP64) is None


def test_batch_iteration_limit(batch):
    probs, b, refs = batch
    rc, results = b.solve(max_iter=3)
    assert rc == condmpc.MAX_ITER
    assert all(r["status"] == condmpc.MAX_ITER and r["iters"] == 3 for r in results)


def test_batch_without_x0_is_rejected(lib):
    probs = ragged_probs()[:2]
    b = condmpc.Batch(probs, with_x0=False)
    with pytest.raises(condmpc.CmpcError) as e:
        b.solve()
    assert e.value.code == condmpc.ERR_INVALID
    b[0].set_x0(probs[0].x0)
    b[1].set_x0(probs[1].x0)
    rc, results = b.solve()
    assert rc == condmpc.OK
    b.close()


def test_batch_of_one_equals_single(lib):
    p = W.heat1d_config("small", instance=3)
    b = condmpc.Batch([p])
    rc, results = b.solve()
    ub, _ = b[0].solution(with_x=False)
    b.close()
    single = condmpc.Problem(p)
    single.set_x0(p.x0)
    r = single.solve()
    us, _ = single.solution(with_x=False)
    single.close()
    assert rc == condmpc.OK and results[0]["iters"] == r["iters"]
    assert np.array_equal(ub, us) and results[0]["obj"] == r["obj"]


def test_batch_instance_errors_name_the_instance(lib):
    probs = ragged_probs()[:3]
    bad = probs[1]
    bad.x0 = bad.x0.copy()
    bad.x0[0] = 0.9  # outside |x| <= xb
    with pytest.raises(condmpc.CmpcError) as e:
        condmpc.Batch(probs)
    assert e.value.code == condmpc.ERR_X0_BOUNDS
    assert "instance 1" in str(e.value)


def test_batch_bf16_start_reaches_the_optimum(batch):
    probs, b, refs = batch
    rc, results = b.solve(precision=condmpc.BF16_SYRK)
    assert rc == condmpc.OK
    for i, (res, ref) in enumerate(zip(results, refs)):
        u, _ = b[i].solution(with_x=False)
        check_against_oracle(f"bf16 {i}", res, ref, u, iters_equal=False)
        assert abs(res["iters"] - ref.iters) <= 4


def test_batch_mixed_equals_single_mixed(batch):
    """The mixed (FP32 start) batch takes the same per-instance decisions as the single path:
    iteration counts, switch iterations and iterates agree bit for bit."""
    probs, b, refs = batch
    rc, results = b.solve(precision=condmpc.FP32_SYRK)
    for i in (0, 4, len(probs) - 1):
        ub, _ = b[i].solution(with_x=False)
        single = condmpc.Problem(probs[i])
        single.set_x0(probs[i].x0)
        r = single.solve(precision=condmpc.FP32_SYRK)
        us, _ = single.solution(with_x=False)
        single.close()
        assert r["iters"] == results[i]["iters"]
        assert r["precision_switch_iter"] == results[i]["precision_switch_iter"]
        assert np.array_equal(ub, us)


def test_batch_rebuilds_views_after_instance_calls(batch):
    """Single solves on instance handles between batch solves: with a tuning-table quantum
    that differs from the batch's, each one rebuilds its instance's SYRK plan (the old plan's
    device memory is freed), and a first BF16 solve allocates the instance's bfloat16 copy of
    Gamma.  The next batch solve at the same precision sees no plan change of its own, so it
    must notice the changed instances and rebuild its device views, work lists and graph; it
    then equals the single solves bit for bit and matches the oracle."""
    probs, b, refs = batch
    condmpc.tune_clear()
    rc, _ = b.solve(precision=condmpc.FP32_SYRK)   # views, lists and graph on the default plans
    assert rc == condmpc.OK
    for i in range(len(probs)):
        for prec in (condmpc.FP32_SYRK, condmpc.BF16_SYRK):
            condmpc.tune_store(b[i].n, b[i].mx, prec, 3000, 1)
    singles = []
    for i in range(len(probs)):
        r = b[i].solve(precision=condmpc.FP32_SYRK)  # re-plans instance i (quantum 3000)
        singles.append((r, b[i].solution(with_x=False)[0]))
    rc, results = b.solve(precision=condmpc.FP32_SYRK)
    assert rc == condmpc.OK
    for i, ((r, us), res, ref) in enumerate(zip(singles, results, refs)):
        ub, _ = b[i].solution(with_x=False)
        assert res["iters"] == r["iters"] and np.array_equal(ub, us), f"instance {i}"
        check_against_oracle(f"replanned {i}", res, ref, ub, iters_equal=False)
    for i in range(len(probs)):
        b[i].solve(precision=condmpc.BF16_SYRK)      # allocates the bfloat16 copy
    rc, results = b.solve(precision=condmpc.BF16_SYRK)
    assert rc == condmpc.OK
    for i, (res, ref) in enumerate(zip(results, refs)):
        ub, _ = b[i].solution(with_x=False)
        check_against_oracle(f"bf16 after singles {i}", res, ref, ub, iters_equal=False)
    condmpc.tune_clear()


def test_batch_warm_starts(batch):
    """cmpc_batch_solve_warm: from given controls every instance takes the oracle's warm
    solve (reading R14) and equals the single-instance warm solve bit for bit; then from each
    instance's last solution shifted one stage."""
    probs, b, refs = batch
    rng = np.random.default_rng(17)
    v0s = [rng.uniform(-0.5, 0.5, p.n) for p in probs]
    rc, results = b.solve_warm([torch.tensor(v, device="cuda") for v in v0s])
    assert rc == condmpc.OK
    ub = [b[i].solution(with_x=False)[0] for i in range(len(probs))]
    for i, (p, res) in enumerate(zip(probs, results)):
        ref = oracle.solve(p, v0=v0s[i])
        check_against_oracle(f"warm {i} {p.name}", res, ref, ub[i])
    for i in (0, 7, 10):  # the single-instance warm start through the same kernels
        single = condmpc.Problem(probs[i])
        single.set_x0(probs[i].x0)
        r = single.solve_warm(v0s[i])
        us, _ = single.solution(with_x=False)
        single.close()
        assert r["iters"] == results[i]["iters"] and np.array_equal(us, ub[i]), f"instance {i}"
    rc, results = b.solve_warm()  # shift of the solution just found
    assert rc == condmpc.OK
    for i, (p, res) in enumerate(zip(probs, results)):
        u, _ = b[i].solution(with_x=False)
        from oracle import condensed_ipm as ipm
        ref = oracle.solve(p, v0=ipm.shift_controls(ub[i], p.nu, p.N))
        check_against_oracle(f"shift {i} {p.name}", res, ref, u, iters_equal=False)
