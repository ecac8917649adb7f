"""Persistent checkpoint of the compressed far coupling (TT cores, eq. (14); ACA factors, eq. (12)):
a handle created without far factors and loaded from a checkpoint gives products bitwise equal to
the handle that wrote it, in both precisions; a checkpoint of the oracle's imported factors
reproduces the oracle's product at the FP64 bar; files for other inputs or options, and damaged
files, are refused without changing the handle."""
import pytest

import vsie_synth as synth
from tests.gpu_common import oracle_same, rel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

E_ARG = 1


@pytest.fixture(scope="module")
def saved(tmp_path_factory):
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    p = synth.small_case()
    op = pkg.Operator(p)
    path = str(tmp_path_factory.mktemp("ckpt") / "small.vsieckpt")
    op.save_checkpoint(path)
    yield p, op, path
    op.close()


def _products(op, seed):
    X = to_dev(synth.complex_normal(op.N, seed, nrhs=2)).reshape(2, op.N)
    return op.matvec(X).clone(), op.matvec(X.to(torch.complex64)).clone()


def test_checkpoint_round_trip_bitwise(saved):
    import paper_2206_12409_amd as pkg
    p, op, path = saved
    ref64, ref32 = _products(op, 51)
    fresh = pkg.Operator(p, build_far=0)
    try:
        before64, _ = _products(fresh, 51)
        assert not torch.equal(before64, ref64)   # no far coupling before the load
        fresh.load_checkpoint(path)
        ranks = lambda o: [[o.sizes.tt_rank[a][k] for k in range(3)] for a in range(3)]
        assert ranks(fresh) == ranks(op)
        assert fresh.sizes.aca_rank == op.sizes.aca_rank
        got64, got32 = _products(fresh, 51)
        assert torch.equal(got64, ref64)
        assert torch.equal(got32, ref32)
        # loading the same file again changes nothing
        fresh.load_checkpoint(path)
        assert torch.equal(_products(fresh, 51)[0], ref64)
    finally:
        fresh.close()


def test_checkpoint_refuses_other_inputs(saved, tmp_path):
    import paper_2206_12409_amd as pkg
    p, op, path = saved
    others = []
    # another seed for the TT-cross index sets and ACA rows
    others.append(pkg.Operator(p, build_far=0, seed=7))
    # another tolerance
    others.append(pkg.Operator(p, build_far=0, tt_tol=2e-3))
    # one voxel of another permittivity
    q = synth.small_case()
    q.grid.eps_r.flat[100] += 1.0
    others.append(pkg.Operator(q, build_far=0))
    try:
        for o in others:
            before = _products(o, 52)[0]
            with pytest.raises(pkg.VsieError) as e:
                o.load_checkpoint(path)
            assert e.value.code == E_ARG
            assert torch.equal(_products(o, 52)[0], before)
    finally:
        for o in others:
            o.close()
    # damaged files: truncated, wrong magic, missing
    raw = open(path, "rb").read()
    bad = [raw[:len(raw) // 2], b"NOTACKPT" + raw[8:]]
    fresh = pkg.Operator(p, build_far=0)
    try:
        before = _products(fresh, 53)[0]
        for i, b in enumerate(bad):
            f = tmp_path / ("bad%d" % i)
            f.write_bytes(b)
            with pytest.raises(pkg.VsieError) as e:
                fresh.load_checkpoint(str(f))
            assert e.value.code == E_ARG
        with pytest.raises(pkg.VsieError):
            fresh.load_checkpoint(str(tmp_path / "missing"))
        assert torch.equal(_products(fresh, 53)[0], before)
    finally:
        fresh.close()


def test_checkpoint_of_oracle_factors_matches_oracle(tmp_path):
    """Factors imported from the oracle, saved, and loaded into a fresh handle: the product of the
    fresh handle matches the oracle's assembled operator with those factors."""
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    p = synth.small_case()
    src = pkg.Operator(p, build_far=0)
    fresh = pkg.Operator(p, build_far=0)
    try:
        d, S_direct, S_same, _ = oracle_same(p, src)
        path = str(tmp_path / "oracle.vsieckpt")
        src.save_checkpoint(path)
        fresh.load_checkpoint(path)
        for seed in (54, 55):
            x = synth.complex_normal(fresh.N, seed)
            y = fresh.matvec(to_dev(x)).cpu().numpy()
            assert rel(y, S_same.matvec(x)) < 1e-10
    finally:
        src.close()
        fresh.close()
