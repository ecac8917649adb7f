"""Oracle of the learned preconditioner's network: a small 3D convolutional U-Net, forward and
backward, in plain NumPy (float64). Test infrastructure only.

Not in the paper (its conclusion, Sec. VI, names a Calderon preconditioner as future work); the
network is the project's addition: it maps the body part of a GMRES residual (three complex field
components as six real channels, plus two channels of the voxel's material coefficient) to a
correction of the body currents.

Layout: activations [D][H][W][C] (z, y, x, channels; channels fastest), grid sizes divisible by 8.
Every convolution is 3 x 3 x 3 with unit stride and zero padding of one voxel ("same"), weights
[Cout][3][3][3][Cin] (taps z, y, x) and a bias per output channel:

    out[z, y, x, o] = b[o] + sum_{dz, dy, dx, i} w[o, dz, dy, dx, i] in[z + dz - 1, y + dy - 1, x + dx - 1, i].

Architecture (level l at 1 / 2^(l-1) of the grid; a leaky ReLU, act(z) = z for z > 0 and
LEAK z otherwise, after every convolution but the last, so that no unit stops learning):

    e1 = conv(conv(x, 8 -> 16), 16 -> 16)              p1 = avgpool2(e1)
    e2 = conv(conv(p1, 16 -> 32), 32 -> 32)            p2 = avgpool2(e2)
    e3 = conv(conv(p2, 32 -> 48), 48 -> 48)            p3 = avgpool2(e3)
    e4 = conv(conv(p3, 48 -> 64), 64 -> 64)
    d3 = conv([up2(e4), e3], 112 -> 48)
    d2 = conv([up2(d3), e2], 80 -> 32)
    d1 = conv([up2(d2), e1], 48 -> 16)
    y  = conv(d1, 16 -> 6)                              (no activation)

avgpool2 is the mean over 2 x 2 x 2 blocks; up2 repeats each voxel into a 2 x 2 x 2 block;
[a, b] concatenates channels (a first). Training minimises the mean squared error
L = sum (y - t)^2 / (2 n), n = the number of target values.

The matrix-core kernels compute in bfloat16 with float32 accumulation; `bf16` below rounds a
float64 array to the nearest bfloat16 (ties to even), so that the oracle can take the same
rounded operands.

Parity pins (tests): the convolution against its definition written as a sum of shifted
products per tap (independent of the einsum layout), adjointness of each layer's backward
(<J v, u> = <v, J^T u> for random v, u), finite-difference gradients of the loss with respect to
every parameter group and the input, pooling and upsampling adjoint to each other up to the
factor 8.
"""
import numpy as np

LEAK = 0.1

LAYERS = (  # (name, Cin, Cout, relu)
    ("e1a", 8, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 32, True), ("e2b", 32, 32, True),
    ("e3a", 32, 48, True), ("e3b", 48, 48, True),
    ("e4a", 48, 64, True), ("e4b", 64, 64, True),
    ("d3", 112, 48, True), ("d2", 80, 32, True), ("d1", 48, 16, True),
    ("out", 16, 6, False),
)


def bf16(a):
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def init_params(seed):
    """He-normal weights (std sqrt(2 / (27 Cin))), zero biases, from numpy's PCG64 (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in LAYERS:
        p[name + ".w"] = rng.standard_normal((co, 3, 3, 3, ci)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)
    return p


def conv3(x, w, b):
    """Forward convolution (definition above): x [D][H][W][Cin], w [Cout][3][3][3][Cin]."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (D, H, W, len(b))).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += xp[dz:dz + D, dy:dy + H, dx:dx + W, :] @ w[:, dz, dy, dx, :].T
    return out


def conv3_backward(x, w, gout):
    """Gradients of sum(gout * conv3(x, w, b)) with respect to x, w and b."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = xp[dz:dz + D, dy:dy + H, dx:dx + W, :]
                gw[:, dz, dy, dx, :] = np.einsum("zyxo,zyxi->oi", gout, win)
                gxp[dz:dz + D, dy:dy + H, dx:dx + W, :] += gout @ w[:, dz, dy, dx, :]
    return gxp[1:-1, 1:-1, 1:-1, :], gw, gout.sum((0, 1, 2))


def avgpool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean((1, 3, 5))


def avgpool2_backward(g):
    return up2(g) / 8.0


def up2(x):
    return x.repeat(2, 0).repeat(2, 1).repeat(2, 2)


def up2_backward(g):
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum((1, 3, 5))


def _identity(a):
    return a


def act(z):
    return np.where(z > 0, z, LEAK * z)


def act_slope(z):
    return np.where(z > 0, 1.0, LEAK)


def forward(p, x, keep=False, quant=False):
    """Network output for input x [D][H][W][8]; with keep, also the activations the backward
    pass needs (pre-activation values of every convolution and its inputs). quant rounds every
    convolution's input and weights to bfloat16 (the matrix-core operands) and keeps the rest in
    float64."""
    acts = {}
    q = bf16 if quant else _identity

    def layer(name, inp, relu):
        z = conv3(q(inp), q(p[name + ".w"]), p[name + ".b"])
        acts[name] = (inp, z)
        return act(z) if relu else z

    e1 = layer("e1b", layer("e1a", x, True), True)
    e2 = layer("e2b", layer("e2a", avgpool2(e1), True), True)
    e3 = layer("e3b", layer("e3a", avgpool2(e2), True), True)
    e4 = layer("e4b", layer("e4a", avgpool2(e3), True), True)
    d3 = layer("d3", np.concatenate([up2(e4), e3], -1), True)
    d2 = layer("d2", np.concatenate([up2(d3), e2], -1), True)
    d1 = layer("d1", np.concatenate([up2(d2), e1], -1), True)
    y = layer("out", d1, False)
    return (y, acts) if keep else y


def loss(p, x, t):
    y = forward(p, x)
    return 0.5 * np.sum((y - t) ** 2) / t.size


def backward(p, x, t, quant=False):
    """Loss and its gradients with respect to every parameter and to the input x. quant: the
    convolutions' operands rounded to bfloat16 as in forward, and in the backward products the
    layer input, the weights and the masked output gradient rounded likewise (the bias gradient
    sums the unrounded output gradient)."""
    y, acts = forward(p, x, keep=True, quant=quant)
    g = {}
    gy = (y - t) / t.size
    q = bf16 if quant else _identity

    def back(name, gout, relu):
        inp, z = acts[name]
        if relu:
            gout = gout * act_slope(z)
        gx, gw, _ = conv3_backward(q(inp), q(p[name + ".w"]), q(gout))
        g[name + ".w"] = gw
        g[name + ".b"] = gout.sum((0, 1, 2))
        return gx

    gd1 = back("out", gy, False)
    gcat1 = back("d1", gd1, True)
    c1 = acts["d1"][0].shape[-1] - 16          # channels of up2(d2) in [up2(d2), e1]
    gd2 = up2_backward(gcat1[..., :c1])
    ge1 = gcat1[..., c1:]
    gcat2 = back("d2", gd2, True)
    c2 = acts["d2"][0].shape[-1] - 32
    gd3 = up2_backward(gcat2[..., :c2])
    ge2 = gcat2[..., c2:]
    gcat3 = back("d3", gd3, True)
    c3 = acts["d3"][0].shape[-1] - 48
    ge4 = up2_backward(gcat3[..., :c3])
    ge3 = gcat3[..., c3:]
    gp3 = back("e4a", back("e4b", ge4, True), True)
    ge3 = ge3 + avgpool2_backward(gp3)
    gp2 = back("e3a", back("e3b", ge3, True), True)
    ge2 = ge2 + avgpool2_backward(gp2)
    gp1 = back("e2a", back("e2b", ge2, True), True)
    ge1 = ge1 + avgpool2_backward(gp1)
    gx = back("e1a", back("e1b", ge1, True), True)
    return 0.5 * np.sum((y - t) ** 2) / t.size, g, gx


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every parameter in place; step counts from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
