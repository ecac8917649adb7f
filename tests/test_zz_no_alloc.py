"""The allocation-free dense solve (vsie_dense_lu_solve_noalloc, static device workspace) against
the allocating entry point vsie_dense_lu_solve, through the C ABI: two calls in a row, the second
with a smaller system, so that the shared workspace's leftover contents from the first call
cannot leak into the second. Same kernels on both sides: the results agree bitwise, and both
agree with a CPU solve within the dense solver's FP64 bar (1e-10 relative, backward error 1e-13)."""
import numpy as np
import pytest

from tests.gpu_common import rel, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_noalloc_dense_solve_matches_allocating_solve():
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    # first a large system with a ragged last panel group, then a smaller one: a stale pivot,
    # permutation entry or singularity flag from the first call would show in the second
    for n, nrhs, seed in ((777, 9, 3), (130, 2, 4)):
        print("noalloc dense solve: n=%d nrhs=%d seed=%d" % (n, nrhs, seed), flush=True)
        A = _rand((n, n), seed)
        B = _rand((n, nrhs), seed + 100)
        A1, B1 = to_dev(A), to_dev(B)
        A2, B2 = to_dev(A), to_dev(B)
        pkg.dense_lu_solve(A1, B1)
        pkg.dense_lu_solve(A2, B2, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(A1, A2) and torch.equal(B1, B2)
        X = B2.cpu().numpy()
        assert rel(X, np.linalg.solve(A, B)) <= 1e-10
        assert np.linalg.norm(A @ X - B) <= 1e-13 * n * np.linalg.norm(A) * np.linalg.norm(X)


def test_noalloc_dense_solve_limits_and_singular():
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    n = pkg.vsie.LU_NOALLOC_MAX_N + 1
    A = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    B = torch.zeros((n, 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(pkg.VsieError) as e:
        pkg.dense_lu_solve(A, B, noalloc=True)
    assert e.value.code == 1
    B = torch.zeros((8, pkg.vsie.LU_NOALLOC_MAX_NRHS + 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(pkg.VsieError) as e:
        pkg.dense_lu_solve(torch.eye(8, dtype=torch.complex128, device="cuda"), B, noalloc=True)
    assert e.value.code == 1
    # an exactly singular matrix reports E_SINGULAR; the next call starts from a cleared flag
    As = _rand((20, 20), 8)
    As[:, 13] = 0
    with pytest.raises(pkg.VsieError) as e:
        pkg.dense_lu_solve(to_dev(As), to_dev(_rand((20, 1), 9)), noalloc=True)
    assert e.value.code == 11
    A = _rand((20, 20), 10)
    B = _rand((20, 1), 11)
    Ad, Bd = to_dev(A), to_dev(B)
    pkg.dense_lu_solve(Ad, Bd, noalloc=True)
    assert rel(Bd.cpu().numpy(), np.linalg.solve(A, B)) <= 1e-10
