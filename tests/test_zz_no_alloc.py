"""cmpc_potrf_noalloc (the factorisation with the library's fixed device scratch) against
cmpc_potrf on the same matrices, through the C ABI: two calls in a row, the second on a
smaller matrix, then a matrix that is not positive definite, then a size above the limit.
The two entry points run the same kernels on the same input, so the factors must agree
bit for bit (and both must be Cholesky factors of the input to 1e-12)."""
import numpy as np
import pytest
import torch

from paper_2209_13049_amd import condmpc

pytestmark = pytest.mark.gpu


def spd(n, seed):
    rng = np.random.default_rng([7, n, seed])
    X = rng.standard_normal((n + 8, n))
    return X.T @ X / n + 0.5 * np.eye(n)


def factor_both(K, ld):
    """Lower factors from cmpc_potrf and cmpc_potrf_noalloc of K (n x n) stored with
    leading dimension ld; entries of the padding and the upper triangle are left alone."""
    n = K.shape[0]
    buf = np.full((n, ld), 7.0)
    buf[:, :n] = K
    a = torch.tensor(buf, device="cuda")
    b = torch.tensor(buf, device="cuda")
    ia = condmpc.potrf(a, ld=ld)
    ib = condmpc.potrf_noalloc(b, ld=ld)
    torch.cuda.synchronize()
    return ia, ib, a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("sizes", [(1000, 130), (333, 64)])
def test_noalloc_matches_potrf_twice(lib, sizes):
    for call, n in enumerate(sizes):
        print(f"[noalloc] call {call}: n = {n}", flush=True)
        K = spd(n, call)
        ld = n + 3
        ia, ib, La, Lb = factor_both(K, ld)
        assert ia == 0 and ib == 0
        assert np.array_equal(La, Lb), f"call {call}, n = {n}"
        L = np.tril(Lb[:, :n])
        err = np.max(np.abs(L @ L.T - K)) / np.max(np.abs(K))
        assert err <= 1e-12, err
        # the strict upper triangle (the input there) and the padding columns are not written
        assert np.all(Lb[:, n:] == 7.0)
        assert np.array_equal(np.triu(Lb[:, :n], 1), np.triu(K, 1))


def test_noalloc_not_positive_definite(lib):
    n = 200
    K = spd(n, 3)
    K[150, 150] = -1.0
    buf_a = torch.tensor(K, device="cuda")
    buf_b = torch.tensor(K, device="cuda")
    with pytest.raises(condmpc.CmpcError) as ea:
        condmpc.potrf(buf_a)
    with pytest.raises(condmpc.CmpcError) as eb:
        condmpc.potrf_noalloc(buf_b)
    assert ea.value.code == eb.value.code == condmpc.ERR_CHOLESKY
    assert str(ea.value) == str(eb.value)
    # the scratch's status flags start from zero at the next call
    K2 = spd(90, 4)
    ia, ib, La, Lb = factor_both(K2, 90)
    assert ia == ib == 0 and np.array_equal(La, Lb)


def test_noalloc_rejects_sizes_above_its_maximum(lib):
    n = condmpc.POTRF_NOALLOC_MAX_N + 1
    K = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
    info = condmpc.ctypes.c_int(0)
    rc = condmpc.load().cmpc_potrf_noalloc(condmpc._dev(K), n, n, condmpc._stream(),
                                            condmpc.ctypes.byref(info))
    assert rc == condmpc.ERR_INVALID
    assert b"exceeds its maximum" in condmpc.load().cmpc_last_error()
