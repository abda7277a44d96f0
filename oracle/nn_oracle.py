"""Plain numpy oracle of the learned Poisson warm start (a small 3D U-Net).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

The paper solves Poisson's equation (Sec. 2.1, Eqs. (3)-(4)) with geometric
multigrid (Sec. 4); it has no network.  This extension predicts an initial
guess for that solve, so the oracle below is the plain definition of each
network operation, written out in FP64 with numpy (one matrix product per
stencil tap), with optional rounding to bfloat16 at the points where the
device path stores bfloat16 tensors.

Tensor layout: [nz][ny][nx][channels] (x fastest among cells, channels
fastest overall).  Conv weights: w[co, dz, dy, dx, ci] for the tap at offset
(dx - 1, dy - 1, dz - 1); zero padding of one cell; bias per output channel.

Architecture for cfg = {"levels": L, "ch": [c0, c1, ...], "cin": 2}:
  encoder level l: e_l = relu(conv(relu(conv(in_l)))) with in_0 = input,
      in_l = pool(e_{l-1}) (mean of 2x2x2 children);
  decoder, l = L-2 .. 0: t = relu(conv_up(d_{l+1})) at level l+1 (c_{l+1} -> c_l),
      s = upsample(t) + e_l (nearest), d_l = relu(conv_dec(s)); d_{L-1} = e_{L-1};
  output: conv_out(d_0), c0 -> 1 channel, no activation.
Parameter order: enc0a, enc0b, enc1a, enc1b, ..., then for l = L-2..0:
  up_l, dec_l; then out; each as weights (co, 3, 3, 3, ci) then bias (co).
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ bfloat16
def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the upper 16 bits of an IEEE binary32; rounding adds
    0x7FFF plus the lowest kept bit before truncation (non-finite values are
    not expected here)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


# ------------------------------------------------------------------- layers
def _pad(x):
    return np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, w, b):
    """y[z, y, x, co] = b[co] + sum over taps and ci of
    x[z + dz - 1, y + dy - 1, x + dx - 1, ci] * w[co, dz, dy, dx, ci]."""
    nz, ny, nx, ci = x.shape
    co = w.shape[0]
    xp = _pad(np.asarray(x, dtype=np.float64))
    y = np.zeros((nz, ny, nx, co)) + np.asarray(b, dtype=np.float64)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = xp[dz:dz + nz, dy:dy + ny, dx:dx + nx, :].reshape(-1, ci)
                y += (sl @ np.asarray(w[:, dz, dy, dx, :], dtype=np.float64).T).reshape(nz, ny, nx, co)
    return y


def conv3d_backward(x, w, dy):
    """Gradients of conv3d: dx (the adjoint, a correlation with the flipped
    taps), dw[co, dz, dy, dx, ci] = sum over cells of x_shifted * dy, db."""
    nz, ny, nx, ci = x.shape
    co = w.shape[0]
    xp = _pad(np.asarray(x, dtype=np.float64))
    dyf = np.asarray(dy, dtype=np.float64).reshape(-1, co)
    dxp = np.zeros_like(xp)
    dw = np.zeros(w.shape)
    for dz in range(3):
        for dy_ in range(3):
            for dx in range(3):
                sl = xp[dz:dz + nz, dy_:dy_ + ny, dx:dx + nx, :].reshape(-1, ci)
                dw[:, dz, dy_, dx, :] = dyf.T @ sl
                dxp[dz:dz + nz, dy_:dy_ + ny, dx:dx + nx, :] += (dyf @ np.asarray(w[:, dz, dy_, dx, :], dtype=np.float64)
                                                                 ).reshape(nz, ny, nx, ci)
    return dxp[1:-1, 1:-1, 1:-1, :], dw, dyf.sum(axis=0)


def pool2(x):
    """Mean over each 2x2x2 block."""
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def up2(x):
    """Nearest-neighbour upsampling by 2 in each direction."""
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------- architecture
def convs(cfg):
    """(name, ci, co) of every convolution in parameter order."""
    L, ch, cin = cfg["levels"], list(cfg["ch"]), cfg.get("cin", 2)
    out = []
    for l in range(L):
        out.append(("enc%da" % l, cin if l == 0 else ch[l - 1], ch[l]))
        out.append(("enc%db" % l, ch[l], ch[l]))
    for l in range(L - 2, -1, -1):
        out.append(("up%d" % l, ch[l + 1], ch[l]))
        out.append(("dec%d" % l, ch[l], ch[l]))
    out.append(("out", ch[0], 1))
    return out


def unpack(params, cfg):
    """Flat parameter vector -> {name: (w, b)}."""
    p = {}
    o = 0
    for name, ci, co in convs(cfg):
        nw = co * 27 * ci
        w = np.asarray(params[o:o + nw], dtype=np.float64).reshape(co, 3, 3, 3, ci)
        o += nw
        b = np.asarray(params[o:o + co], dtype=np.float64)
        o += co
        p[name] = (w, b)
    assert o == len(params), "parameter count does not match the architecture"
    return p


def n_params(cfg):
    return sum(co * 27 * ci + co for _, ci, co in convs(cfg))


# ------------------------------------------------------------ forward/back
def forward(params, x, cfg, rounding=True):
    """Network output and the cache for backward.  With rounding, the input,
    the weights (not the biases) and every stored activation are rounded to
    bfloat16 where the device stores them; the output stays FP32."""
    R = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    L = cfg["levels"]
    P = unpack(params, cfg)
    Wq = {k: (R(w), np.asarray(b, dtype=np.float64)) for k, (w, b) in P.items()}
    cache = {"in": R(x)}
    cur = cache["in"]
    for l in range(L):
        if l > 0:
            cur = R(pool2(cache["e%d" % (l - 1)]))
            cache["p%d" % l] = cur
        w, b = Wq["enc%da" % l]
        a = R(relu(conv3d(cur, w, b)))
        cache["a%d" % l] = a
        w, b = Wq["enc%db" % l]
        cache["e%d" % l] = R(relu(conv3d(a, w, b)))
    d = cache["e%d" % (L - 1)]
    for l in range(L - 2, -1, -1):
        cache["d%d" % (l + 1)] = d
        w, b = Wq["up%d" % l]
        t = R(relu(conv3d(d, w, b)))
        cache["t%d" % l] = t
        s = R(up2(t) + cache["e%d" % l])
        cache["s%d" % l] = s
        w, b = Wq["dec%d" % l]
        d = R(relu(conv3d(s, w, b)))
    cache["d0"] = d
    w, b = Wq["out"]
    out = conv3d(d, w, b)
    if rounding:
        out = f32(out)
    cache["W"] = Wq
    return out, cache


def backward(params, cache, dout, cfg, grad_rounding=False):
    """Gradient of sum(out * dout) with respect to the flat parameters (the
    forward's rounding points are treated as identities, as in training).
    With grad_rounding the output gradient of each convolution is rounded to
    bfloat16 where it feeds the input-gradient product (the device path runs
    that product on bfloat16 operands); weight gradients use it unrounded."""
    L = cfg["levels"]
    W = cache["W"]
    g = {}

    def conv3d_backward(x, w, dy):
        dx = _conv_dx(w, bf16(dy) if grad_rounding else dy, x.shape)
        _, dw, db = _conv3d_backward(x, w, dy)
        return dx, dw, db

    w, _ = W["out"]
    dd, dw, db = conv3d_backward(cache["d0"], w, dout)
    g["out"] = (dw, db)
    de = {}
    for l in range(0, L - 1):
        # d_l = relu(conv_dec(s_l)): mask by the stored activation
        dd = dd * (cache["d0"] > 0) if l == 0 else dd * (cache["d%d" % l] > 0)
        w, _ = W["dec%d" % l]
        ds, dw, db = conv3d_backward(cache["s%d" % l], w, dd)
        g["dec%d" % l] = (dw, db)
        de[l] = ds                                   # skip branch
        dt = pool2(ds) * 8.0                         # adjoint of nearest upsampling
        dt = dt * (cache["t%d" % l] > 0)
        w, _ = W["up%d" % l]
        dd, dw, db = conv3d_backward(cache["d%d" % (l + 1)], w, dt)
        g["up%d" % l] = (dw, db)
    # dd is now the gradient of d_{L-1} = e_{L-1}
    acc = {L - 1: dd}
    for l in range(L - 1, -1, -1):
        ge = acc[l] + de.get(l, 0.0) if l < L - 1 else acc[l]
        ge = ge * (cache["e%d" % l] > 0)
        w, _ = W["enc%db" % l]
        da, dw, db = conv3d_backward(cache["a%d" % l], w, ge)
        g["enc%db" % l] = (dw, db)
        da = da * (cache["a%d" % l] > 0)
        w, _ = W["enc%da" % l]
        src = cache["in"] if l == 0 else cache["p%d" % l]
        dp, dw, db = conv3d_backward(src, w, da)
        g["enc%da" % l] = (dw, db)
        if l > 0:
            acc[l - 1] = up2(dp) / 8.0               # adjoint of the 2x2x2 mean
    flat = []
    for name, _, _ in convs(cfg):
        dw, db = g[name]
        flat.append(dw.ravel())
        flat.append(db.ravel())
    return np.concatenate(flat)


_conv3d_backward = conv3d_backward


def _conv_dx(w, dy, xshape):
    return conv3d_backward(np.zeros(xshape), w, dy)[0]


def mse(out, target):
    """Mean squared error and its gradient with respect to out."""
    d = np.asarray(out, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) with bias correction; t counts
    from 1."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- features
def features(rho, grid, bc, eps0):
    """Network input of the warm start and its scale: channel 0 is
    rho * Lx^2 / (eps0 * V), channel 1 the electrode ramp / V, where the ramp
    is the linear interpolation between the Dirichlet values of the x faces
    (the Laplace solution for two plates with zero-flux side walls, the
    configuration of the streamer runs), and V = max |Dirichlet value|
    (1 if all are 0).  The solution guess is V times the output."""
    nx, ny, nz, dx, dy, dz = grid
    kinds, vals = list(bc["kind"]), list(bc["value"])
    dvals = [abs(vals[f]) for f in range(6) if kinds[f] == 0]
    V = max(dvals) if dvals and max(dvals) > 0 else 1.0
    Lx = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    if kinds[0] == 0 and kinds[1] == 0:
        ramp = vals[0] + (vals[1] - vals[0]) * xc / Lx
    else:
        ramp = np.zeros(nx)
    f = np.zeros((nz, ny, nx, 2))
    f[..., 0] = np.asarray(rho, dtype=np.float64) * Lx * Lx / (eps0 * V)
    f[..., 1] = np.broadcast_to(ramp / V, (nz, ny, nx))
    return f, V
