"""The graph-replayed product (vsie_matvec_graph) against the plain one, bit for bit: several
replays with the program's own eager work and synchronisations between them, several buffer pairs
(one graph each), several columns and both precisions; and against the oracle at the FP64 bar."""
import numpy as np
import pytest

import vsie_synth as synth
from tests.gpu_common import oracle_same, rel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def small():
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    p = synth.small_case()
    op = pkg.Operator(p)
    yield p, op
    op.close()


@pytest.mark.parametrize("dtype,nrhs", [(torch.complex128, 1), (torch.complex128, 3), (torch.complex64, 2)])
def test_graph_replays_match_eager(small, dtype, nrhs):
    p, op = small
    X = to_dev(synth.complex_normal(op.N, 31, nrhs=nrhs), dtype).reshape(nrhs, op.N)
    Y = torch.empty_like(X)
    ref = op.matvec(X).clone()
    other = to_dev(synth.complex_normal(op.N, 32), dtype)
    for rep in range(4):
        Y.fill_(float("nan"))
        op.matvec_graph(X, Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), "replay %d" % rep
        # eager work of the program between replays: other products and a host round trip
        op.matvec(other)
        _ = float(torch.linalg.vector_norm(other).item())
        torch.cuda.synchronize()
    # a new input in the same buffer is seen by the replay
    X2 = to_dev(synth.complex_normal(op.N, 33, nrhs=nrhs), dtype).reshape(nrhs, op.N)
    X.copy_(X2)
    op.matvec_graph(X, Y)
    assert torch.equal(Y, op.matvec(X2))


def test_graph_second_buffer_pair_and_oracle(small):
    """Two buffer pairs, each with its graph; a graph captured before vsie_import replaced the
    compressed factors is not replayed afterwards (the import drops the cached graphs)."""
    p, op = small
    xs = [synth.complex_normal(op.N, s) for s in (41, 42)]
    X = [to_dev(x) for x in xs]
    Y = [torch.empty_like(x) for x in X]
    op.matvec_graph(X[0], Y[0])   # captured with the library's own TT and ACA factors
    torch.cuda.synchronize()
    d, S_direct, S_same, _ = oracle_same(p, op)   # imports the oracle's factors
    for _ in range(2):
        for x, y in zip(X, Y):
            op.matvec_graph(x, y)
    torch.cuda.synchronize()
    for x, y in zip(xs, Y):
        assert rel(y.cpu().numpy(), S_same.matvec(x)) < 1e-10
