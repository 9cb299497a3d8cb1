"""Ragged batches at the sizes of the configured batch workload (ns up to ~1900, nu up to 16,
N up to 64: K up to 960 x 960, 15 tile columns), a few instances at a time.

The small ragged batch of the other batch tests stays within three tile columns; these
instances reach the batch forms that only larger K use: the Cholesky step lists for k up to
14 with their fused forward-substitution items, the one-workgroup solve in its pipelined form
(4 to 8 block steps) and its looped form (more than 8), and state dimensions up to ~1900 in the
Gamma pass lists.

* FP64: every instance converges and equals its single-instance solve bit for bit (same
  iterates, same iteration count); two instances (9 and 12 tile columns) meet the oracle's bar;
* FP32 start (default plans, no tuning): every instance converges to the FP64 batch's optimum
  within the solve tolerance;
* the benchmarked workload as a batch on the autotuner's FP64 plan equals single solves on the
  same plan bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu

# instances of batch_instances(96, seed=21): (index, tile columns)
PICK = [(63, 1), (7, 4), (2, 5), (8, 9), (12, 12), (69, 13), (30, 15)]
ORACLE = (8, 12)  # n = 520 (ns 1752, 91,104 state rows) and n = 720 (ns 354)


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.fixture(scope="module")
def large(lib):
    allp = W.batch_instances(96, seed=21)
    probs = []
    for i, nt in PICK:
        p = allp[i]
        assert (p.n + 63) // 64 == nt
        probs.append(p)
    print("[batch-large] sizes " + ", ".join(f"(ns {p.ns}, n {p.n})" for p in probs), flush=True)
    b = condmpc.Batch(probs)
    yield probs, b
    b.close()


def test_large_batch_fp64_bitwise_single_and_oracle(large):
    probs, b = large
    rc, results = b.solve(precision=condmpc.FP64)
    print(f"[batch-large] fp64: rc {rc}, iters {[r['iters'] for r in results]}", flush=True)
    assert rc == condmpc.OK
    for j, ((i, nt), p, res) in enumerate(zip(PICK, probs, results)):
        assert res["status"] == condmpc.OK, f"instance {i}"
        assert res["primal_res"] <= 1e-8 and res["dual_res"] <= 1e-8 and res["compl_res"] <= 1e-8
        ub, _ = b[j].solution(with_x=False)
        vb, sb, lb, zb = b[j].iterate()
        single = condmpc.Problem(p)
        single.set_x0(p.x0)
        r = single.solve()
        us, _ = single.solution(with_x=False)
        vs, ss, ls, zs = single.iterate()
        single.close()
        print(f"[batch-large] {i} (nt {nt}): batch iters {res['iters']} single {r['iters']} "
              f"obj {res['obj']:.12e}", flush=True)
        assert r["iters"] == res["iters"], f"instance {i}"
        assert np.array_equal(ub, us), f"instance {i}: u differs"
        assert np.array_equal(sb, ss) and np.array_equal(lb, ls) and np.array_equal(zb, zs)
        if i in ORACLE:
            ref = oracle.solve(p)
            print(f"[batch-large] {i}: oracle iters {ref.iters} obj {ref.obj:.12e}", flush=True)
            assert ref.status == oracle.STATUS_CONVERGED
            assert res["iters"] == ref.iters
            assert abs(res["obj"] - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))
            assert rel_err(ub, ref.v) <= 1e-6


def test_large_batch_fp32_start_reaches_the_optimum(large):
    probs, b = large
    rc, r64 = b.solve(precision=condmpc.FP64)
    assert rc == condmpc.OK
    u64 = [b[j].solution(with_x=False)[0] for j in range(len(probs))]
    rc, r32 = b.solve(precision=condmpc.FP32_SYRK)
    print(f"[batch-large] fp32: rc {rc}, iters {[r['iters'] for r in r32]}, switch "
          f"{[r['precision_switch_iter'] for r in r32]}", flush=True)
    assert rc == condmpc.OK
    for j, (a, c) in enumerate(zip(r32, r64)):
        assert a["status"] == condmpc.OK, f"instance {PICK[j][0]}"
        assert a["primal_res"] <= 1e-8 and a["dual_res"] <= 1e-8 and a["compl_res"] <= 1e-8
        assert abs(a["obj"] - c["obj"]) <= 1e-8 * max(1.0, abs(c["obj"]))
        assert abs(a["iters"] - c["iters"]) <= 3
        u, _ = b[j].solution(with_x=False)
        assert rel_err(u, u64[j]) <= 1e-6


def test_headline_batch_tuned_fp64_bitwise_single(lib):
    """Four instances of the benchmarked workload (K 500 x 500, 50,000 state rows): the
    autotuner's FP64 plan, then the batch against single solves that follow the same tuning
    entry, bit for bit; the table is cleared afterwards."""
    probs = [W.heat1d_config("1d", instance=k) for k in range(4)]
    condmpc.tune_clear()
    b = condmpc.Batch(probs)
    try:
        rep = b.tune(condmpc.FP64)
        print(f"[batch-large] headline tune: {rep}", flush=True)
        assert rep["quantum"] in (3000, 6000, 12000, 24000, 48000, 96000)
        rc, results = b.solve(precision=condmpc.FP64)
        assert rc == condmpc.OK
        for j, p in enumerate(probs):
            assert condmpc.tune_lookup(p.n, b[j].mx, condmpc.FP64) == (rep["quantum"],
                                                                      rep["persistent"])
            ub, _ = b[j].solution(with_x=False)
            single = condmpc.Problem(p)
            single.set_x0(p.x0)
            r = single.solve()
            us, _ = single.solution(with_x=False)
            single.close()
            assert results[j]["status"] == condmpc.OK and r["iters"] == results[j]["iters"]
            assert np.array_equal(ub, us), f"instance {j}"
    finally:
        b.close()
        condmpc.tune_clear()
