"""GPU parity of the learned preconditioner's network kernels (bfloat16 matrix-core convolutions,
float32 accumulation) against the oracle (oracle/cnn.py) taking the same bfloat16-rounded operands:
single layers forward, backward-data and weight gradient on a ragged grid (tiles of 16 x 4 voxels
cut at the edges), the whole network's forward and gradients, and the Adam step.

Bars: a single layer 2e-5 relative to its largest output (float32 accumulation of up to 3024
products); the whole network's output 2e-3 and its gradients 8e-3 per parameter group, four
bfloat16 unit roundoffs (2^-9 each): activations between layers are float32 on the device and
float64 in the oracle, so the next layer's bfloat16 rounding of a value can differ by one unit,
and the gradients pass through twelve such roundings twice; Adam 1e-6 relative."""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2206_12409_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return pkg


def _pad(a, cp):
    out = np.zeros(a.shape[:-1] + (cp,), np.float32)
    out[..., :a.shape[-1]] = a
    return torch.from_numpy(out).cuda()


def _cp(c):
    return (c + 15) // 16 * 16


def _relerr(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def net(lib):
    n = lib.Net(seed=5)
    rng = np.random.default_rng(9)
    p = lib.Net.unflatten(n.get_params().copy())
    for k in p:
        if k.endswith(".b"):
            p[k][:] = 0.1 * rng.standard_normal(p[k].shape)
    n.set_params(lib.Net.flatten(p))
    pf = lib.Net.unflatten(n.get_params().astype(np.float64))
    return n, pf


DIMS = (4, 6, 18)   # z, y, x: ragged against the 16 x 4 tiles


@pytest.mark.parametrize("layer", [0, 2, 7, 8, 10, 11])
def test_layer_forward_and_backward_data(net, lib, layer):
    n, p = net
    name, ci, co, relu = lib.vsie.NET_LAYERS[layer]
    rng = np.random.default_rng(layer)
    D, H, W = DIMS
    dec = 8 <= layer <= 10
    cb = {8: 48, 9: 32, 10: 16}.get(layer, 0)
    w, b = p[name + ".w"], p[name + ".b"]
    if dec:
        a = rng.standard_normal((D // 2, H // 2, W // 2, ci - cb)).astype(np.float32)
        s = rng.standard_normal((D, H, W, cb)).astype(np.float32)
        x = np.concatenate([cnn.up2(a.astype(np.float64)), s.astype(np.float64)], -1)
        in0, in1 = _pad(a, ci - cb), _pad(s, cb)
    else:
        x = rng.standard_normal((D, H, W, ci)).astype(np.float32).astype(np.float64)
        in0, in1 = _pad(x, _cp(ci)), None
    out = torch.empty((D, H, W, _cp(co)), dtype=torch.float32, device="cuda")
    n.layer(layer, 0, DIMS, in0, in1, None, out)
    z = cnn.conv3(cnn.bf16(x), cnn.bf16(w), b)
    ref = cnn.act(z) if relu else z
    got = out.cpu().numpy()
    e = _relerr(got[..., :co], ref)
    print("layer %s forward: %.2e" % (name, e))
    assert e < 2e-5
    assert np.all(got[..., co:] == 0)
    # backward-data: gradient of the layer input from a random output gradient, ReLU-masked
    g = rng.standard_normal((D, H, W, co)).astype(np.float32).astype(np.float64)
    gm = g * cnn.act_slope(ref) if relu else g
    gx_ref, _, _ = cnn.conv3_backward(cnn.bf16(x), cnn.bf16(w), cnn.bf16(gm))
    gout = torch.empty((D, H, W, _cp(ci) if not dec else ci), dtype=torch.float32, device="cuda")
    n.layer(layer, 1, DIMS, _pad(g, _cp(co)), None, out if relu else None, gout)
    gx = gout.cpu().numpy()
    e = _relerr(gx[..., :ci], gx_ref)
    print("layer %s backward-data: %.2e" % (name, e))
    assert e < 2e-5


@pytest.mark.parametrize("layer", [0, 3, 8, 11])
def test_layer_weight_gradient(net, lib, layer):
    n, p = net
    name, ci, co, relu = lib.vsie.NET_LAYERS[layer]
    rng = np.random.default_rng(100 + layer)
    D, H, W = DIMS
    dec = 8 <= layer <= 10
    cb = {8: 48, 9: 32, 10: 16}.get(layer, 0)
    if dec:
        a = rng.standard_normal((D // 2, H // 2, W // 2, ci - cb)).astype(np.float32)
        s = rng.standard_normal((D, H, W, cb)).astype(np.float32)
        x = np.concatenate([cnn.up2(a.astype(np.float64)), s.astype(np.float64)], -1)
        in0, in1 = _pad(a, ci - cb), _pad(s, cb)
    else:
        x = rng.standard_normal((D, H, W, ci)).astype(np.float32).astype(np.float64)
        in0, in1 = _pad(x, _cp(ci)), None
    g = rng.standard_normal((D, H, W, co)).astype(np.float32).astype(np.float64)
    mask = rng.standard_normal((D, H, W, co)).astype(np.float32) if relu else None
    gm = g * cnn.act_slope(mask) if relu else g
    _, gw_ref, _ = cnn.conv3_backward(cnn.bf16(x), cnn.bf16(p[name + ".w"]), cnn.bf16(gm))
    gb_ref = gm.sum((0, 1, 2))
    gw, gb = n.layer_wgrad(layer, DIMS, in0, _pad(g, _cp(co)), in1, _pad(mask, _cp(co)) if relu else None)
    e = _relerr(gw, gw_ref)
    eb = _relerr(gb, gb_ref)
    print("layer %s weight gradient %.2e, bias gradient %.2e" % (name, e, eb))
    assert e < 2e-5 and eb < 2e-5


def test_network_forward_and_gradients(net, lib):
    n, p = net
    rng = np.random.default_rng(21)
    x = rng.standard_normal((8, 8, 16, 8)).astype(np.float32)
    t = rng.standard_normal((8, 8, 16, 6)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    y = n.forward(xd).cpu().numpy()
    y_ref = cnn.forward(p, x.astype(np.float64), quant=True)
    e = float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))
    print("network forward: %.2e" % e)
    assert e < 2e-3
    L, gflat = n.gradients(xd, td)
    L_ref, g_ref, _ = cnn.backward(p, x.astype(np.float64), t.astype(np.float64), quant=True)
    assert abs(L - L_ref) < 2e-3 * L_ref
    g = lib.Net.unflatten(gflat)
    worst = max(float(np.linalg.norm(g[k] - g_ref[k]) / np.linalg.norm(g_ref[k])) for k in g_ref)
    print("network gradients: worst parameter group %.2e" % worst)
    assert worst < 8e-3


def test_adam_step_matches_oracle(lib):
    n = lib.Net(seed=3)
    rng = np.random.default_rng(22)
    x = torch.from_numpy(rng.standard_normal((8, 8, 8, 8)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((8, 8, 8, 6)).astype(np.float32)).cuda()
    p0 = n.get_params().astype(np.float64)
    pd = {"all": p0.copy()}
    m = {"all": np.zeros_like(p0)}
    v = {"all": np.zeros_like(p0)}
    for step in range(1, 4):
        _, g = n.gradients(x, t)
        n.adam(1e-3)
        cnn.adam_step(pd, {"all": g.astype(np.float64)}, m, v, step, 1e-3)
        got = n.get_params().astype(np.float64)
        assert np.abs(got - pd["all"]).max() <= 1e-6 * np.abs(pd["all"]).max() + 1e-9
        pd["all"] = got   # follow the device's parameters (the next gradients are taken there)
