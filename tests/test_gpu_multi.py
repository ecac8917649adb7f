"""Several phantoms inside one shield: operators built with vsie_create_shared use the donor's
dense far block (results bit for bit those of an operator that assembled its own, in any
destruction order; a different shield is refused), and the products of operators with uneven grids
run from one captured graph with the results of the separate products, bit for bit, on every
replay."""
import numpy as np
import pytest

import vsie_synth as synth
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem(n, shield, loop):
    g = synth.sphere_phantom(n, 5e-3, 17e-3, 52.0, 0.55)
    return synth.Problem(g, [shield, loop], synth.problems.LARMOR_7T_HZ, "n%s" % (n,))


@pytest.fixture(scope="module")
def parts():
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    base = synth.small_case()
    shield, loop = base.meshes
    return pkg, shield, loop


def test_shared_far_block_and_graph(parts):
    pkg, shield, loop = parts
    pa, pb = _problem((8, 8, 8), shield, loop), _problem((9, 8, 10), shield, loop)
    A = pkg.Operator(pa)
    B = pkg.Operator(pb, share_far_with=A)
    B_own = pkg.Operator(pb)
    assert B.N == B_own.N
    xb = to_dev(synth.complex_normal(B.N, 51))
    yb = B.matvec(xb).clone()
    assert torch.equal(yb, B_own.matvec(xb))
    B_own.close()
    # one graph for both operators (different grids), replayed with eager work between
    xa = to_dev(synth.complex_normal(A.N, 52))
    ya_ref = A.matvec(xa).clone()
    oa, ob = torch.empty_like(xa), torch.empty_like(xb)
    G = pkg.ProductGraph([A, B], [xa, xb], [oa, ob])
    for rep in range(3):
        oa.fill_(float("nan"))
        ob.fill_(float("nan"))
        G.launch()
        torch.cuda.synchronize()
        assert torch.equal(oa, ya_ref) and torch.equal(ob, yb), "replay %d" % rep
        A.matvec(xa)   # eager work of the program between replays
        torch.cuda.synchronize()
    G.close()
    # the donor goes first; the sharer keeps the block
    A.close()
    assert torch.equal(B.matvec(xb), yb)
    B.close()


def test_shared_far_block_refuses_other_shield(parts):
    pkg, shield, loop = parts
    other = synth.meshes.cylinder_shield(0.085, 0.160, 12, 6, closed=True, cap_rings=2)
    A = pkg.Operator(_problem((8, 8, 8), shield, loop))
    with pytest.raises(pkg.VsieError):
        pkg.Operator(_problem((8, 8, 8), other, loop), share_far_with=A)
    A.close()


def test_graph_complex64_uneven_grids(parts):
    pkg, shield, loop = parts
    ops = [pkg.Operator(_problem(n, shield, loop)) for n in ((8, 8, 8), (10, 9, 8))]
    xs = [to_dev(synth.complex_normal(op.N, 60 + i, nrhs=2), torch.complex64).reshape(2, op.N)
          for i, op in enumerate(ops)]
    refs = [op.matvec(x).clone() for op, x in zip(ops, xs)]
    outs = [torch.empty_like(x) for x in xs]
    G = pkg.ProductGraph(ops, xs, outs)
    for _ in range(2):
        G.launch()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
    G.close()
    for op in ops:
        op.close()
