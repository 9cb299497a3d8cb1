"""The Cholesky factorisation and the triangular solves of Section 3 on ill-conditioned condensed
matrices: the matrices K of the last iterations of Algorithm 1 on the general-data heat workload
with three 64-column tiles (condition numbers up to ~1e13; diagonal factor tiles with
max|L_kk| max|L_kk^-1| up to ~3e5), taken from the oracle's own solve.  A factorisation and a
solve by substitution are backward stable on them; the library's, which work with the inverses
of the diagonal tiles, must be too (they refine where a tile is ill-conditioned).  Without that
refinement the factorisation broke down on these matrices and the solves had backward errors up
to ~1e-10."""
import numpy as np
import pytest
import torch

import oracle
from paper_2209_13049_amd import condmpc
from paper_2209_13049_amd import workloads as W

pytestmark = pytest.mark.gpu

ITERS = (10, 12, 13, 15)  # late iterations, where the tiles are the most ill-conditioned


@pytest.fixture(scope="module")
def matrices():
    p = W.heat1d_general(90, 9, 16, kgain=0.3)
    log = []
    r = oracle.solve(p, callback=log.append)
    assert r.status == oracle.STATUS_CONVERGED and r.iters > max(ITERS)
    out = {}
    for it in ITERS:
        K = np.tril(log[it]["K"])
        out[it] = K + np.tril(K, -1).T
    return out


@pytest.mark.parametrize("it", ITERS)
def test_potrf_potrs_backward_stable(lib, matrices, it):
    K = matrices[it]
    n = K.shape[0]
    cond = np.linalg.cond(K)
    Kt = torch.tensor(K, device="cuda")
    condmpc.potrf(Kt)
    L = np.tril(Kt.cpu().numpy())
    bw = np.max(np.abs(L @ L.T - K)) / np.max(np.abs(K))
    b = np.random.default_rng(it).normal(size=n)
    bt = torch.tensor(b, device="cuda")
    condmpc.potrs(Kt, bt)
    x = bt.cpu().numpy()
    sbw = np.linalg.norm(K @ x - b) / (np.linalg.norm(K, 2) * np.linalg.norm(x))
    print(f"[chol] iteration {it}: cond {cond:.1e} factor backward error {bw:.1e} "
          f"solve backward error {sbw:.1e}", flush=True)
    assert cond > 1e9
    assert bw <= 64 * np.finfo(float).eps
    assert sbw <= 64 * np.finfo(float).eps
