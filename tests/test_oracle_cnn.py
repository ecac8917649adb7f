"""Pins of the learned preconditioner's network oracle (oracle/cnn.py): the convolution against
its definition written voxel by voxel, adjoint identities of every backward piece, finite
differences of the loss for every parameter group and the input, bfloat16 rounding and the Adam
step against library routines."""
import numpy as np
import pytest

from oracle import cnn


def _conv_by_definition(x, w, b):
    D, H, W, Ci = x.shape
    out = np.zeros((D, H, W, w.shape[0]))
    for z in range(D):
        for y in range(H):
            for xx in range(W):
                acc = b.copy()
                for dz in range(3):
                    for dy in range(3):
                        for dx in range(3):
                            zz, yy, x3 = z + dz - 1, y + dy - 1, xx + dx - 1
                            if 0 <= zz < D and 0 <= yy < H and 0 <= x3 < W:
                                acc = acc + w[:, dz, dy, dx, :] @ x[zz, yy, x3, :]
                out[z, y, xx] = acc
    return out


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 3))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    assert np.allclose(cnn.conv3(x, w, b), _conv_by_definition(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 6, 5))
    w = rng.standard_normal((3, 3, 3, 3, 5))
    u = rng.standard_normal((4, 4, 6, 3))
    gx, gw, gb = cnn.conv3_backward(x, w, u)
    zero = np.zeros(3)
    v = rng.standard_normal(x.shape)
    assert np.isclose(np.sum(cnn.conv3(v, w, zero) * u), np.sum(v * gx), rtol=1e-12)
    dw = rng.standard_normal(w.shape)
    assert np.isclose(np.sum(cnn.conv3(x, dw, zero) * u), np.sum(dw * gw), rtol=1e-12)
    db = rng.standard_normal(3)
    assert np.isclose(np.sum((cnn.conv3(x, w, db) - cnn.conv3(x, w, zero)) * u), np.sum(db * gb), rtol=1e-12)


def test_pool_and_upsample_adjoint():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 6, 8, 3))
    c = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(cnn.avgpool2(a) * c), np.sum(a * cnn.up2(c)) / 8.0, rtol=1e-13)
    assert np.isclose(np.sum(cnn.up2(c) * a), np.sum(c * cnn.up2_backward(a)), rtol=1e-13)
    assert np.allclose(cnn.avgpool2_backward(c), cnn.up2(c) / 8.0)
    # averaging then repeating reproduces a field that is constant on 2 x 2 x 2 blocks
    assert np.allclose(cnn.avgpool2(cnn.up2(c)), c)


@pytest.fixture(scope="module")
def net_case():
    rng = np.random.default_rng(3)
    p = cnn.init_params(7)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((8, 8, 16, 8))
    t = rng.standard_normal((8, 8, 16, 6))
    return p, x, t


def test_loss_gradients_by_finite_differences(net_case):
    """Central differences along a random direction of each parameter group and of the input
    agree with the backward pass (ReLU kinks are met with probability zero)."""
    p, x, t = net_case
    L, g, gx = cnn.backward(p, x, t)
    assert np.isclose(L, cnn.loss(p, x, t), rtol=1e-14)
    rng = np.random.default_rng(4)
    eps = 1e-7   # small enough that no ReLU of the first layers changes sign inside the stencil
    for k in p:
        d = rng.standard_normal(p[k].shape)
        pp = dict(p)
        pm = dict(p)
        pp[k] = p[k] + eps * d
        pm[k] = p[k] - eps * d
        fd = (cnn.loss(pp, x, t) - cnn.loss(pm, x, t)) / (2 * eps)
        an = np.sum(g[k] * d)
        assert abs(fd - an) <= 2e-6 * max(abs(an), 1e-8), (k, fd, an)
    d = rng.standard_normal(x.shape)
    fd = (cnn.loss(p, x + eps * d, t) - cnn.loss(p, x - eps * d, t)) / (2 * eps)
    assert abs(fd - np.sum(gx * d)) <= 2e-6 * abs(fd)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.uniform(-20, 20, 10000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -(1.0 + 2.0 ** -8), 0.0, 65504.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(a), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert cnn.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0


def test_adam_step_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    p = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    tp = {k: torch.tensor(w, requires_grad=True) for k, w in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-2)
    for step in range(1, 4):
        g = {k: rng.standard_normal(w.shape) for k, w in p.items()}
        cnn.adam_step(p, g, m, v, step, 1e-2)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)
