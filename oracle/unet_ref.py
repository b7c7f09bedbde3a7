"""FP64 reference of the warm-start U-Net and of its lattice <-> network fields.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never does, and it shares
no code with the GPU library.

The network is not part of the paper (which starts every run from the
profile of Eq. 16); it is the learned warm start that replaces that profile.
Every layer here is its textbook definition in float64 numpy, written as a
loop over kernel taps or window positions with whole-array slices inside:

* 3x3 convolution with zero padding 1 (cross-correlation, no kernel flip):
  y[n, h, w, o] = b[o] + sum_{dy, dx, i} x[n, h + dy, w + dx, i] W[o, dy + 1, dx + 1, i];
* ReLU; 2x2 max pooling with stride 2 (the first maximum in the order
  (0, 0), (0, 1), (1, 0), (1, 1) receives the gradient);
* 2x2 stride-2 transposed convolution:
  y[n, 2h + a, 2w + b, o] = bias[o] + sum_i x[n, h, w, i] W[a, b, o, i];
* skip connections by channel concatenation [upsampled | encoder output];
* 1x1 head to one channel; mean squared error.

Backward passes are the chain rule of those definitions.  The flat
parameter order is the one the C interface documents for
lbm_unet_get_params.

ReLU masks and pooling choices are discrete decisions taken on forward
values.  With storage="bf16" the forward pass rounds, as the GPU network
stores them, the input, the convolution weights and every activation to
bfloat16 (round to nearest even; all arithmetic stays float64), so that both
sides take those decisions on the same values; gradients are never rounded.

Pins (tests/test_oracle_unet.py): the convolution against
scipy.signal.correlate2d, tap convention with a delta kernel, the
transposed convolution as the adjoint of its data gradient and against
explicit loops, pooling against brute force, every gradient against central
finite differences of the loss, the first Adam step against its closed form,
and the warm-start density against an independent root finder.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------
def conv3x3(x, w, b):
    """x [n,H,W,Ci], w [Co,3,3,Ci], b [Co] -> [n,H,W,Co]."""
    n, H, W, _ = x.shape
    xp = np.zeros((n, H + 2, W + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, H, W, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    return y


def conv3x3_bwd(x, w, gy):
    """Gradients of conv3x3 with respect to x, w and b, given dL/dy."""
    n, H, W, Ci = x.shape
    xp = np.zeros((n, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    g2 = gy.reshape(-1, gy.shape[3])
    for ky in range(3):
        for kx in range(3):
            gxp[:, ky:ky + H, kx:kx + W, :] += gy @ w[:, ky, kx, :]
            gw[:, ky, kx, :] = g2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, Ci)
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(0, 1, 2))


def relu(z):
    return np.maximum(z, 0.0)


def maxpool2(x):
    """2x2 max pooling; returns the pooled tensor and the window position of the first maximum."""
    n, H, W, C = x.shape
    win = np.stack([x[:, a::2, b::2, :][:, :H // 2, :W // 2] for a in (0, 1) for b in (0, 1)])
    return win.max(axis=0), win.argmax(axis=0)


def maxpool2_bwd(shape, arg, gy):
    gx = np.zeros(shape)
    for k, (a, b) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        gx[:, a::2, b::2, :][:, :gy.shape[1], :gy.shape[2]] += np.where(arg == k, gy, 0.0)
    return gx


def upconv2(x, w, b):
    """x [n,H,W,Ci], w [2,2,Co,Ci], b [Co] -> [n,2H,2W,Co]."""
    n, H, W, _ = x.shape
    y = np.empty((n, 2 * H, 2 * W, w.shape[2]))
    for a in (0, 1):
        for c in (0, 1):
            y[:, a::2, c::2, :] = x @ w[a, c].T + b
    return y


def upconv2_bwd(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    x2 = x.reshape(-1, x.shape[3])
    for a in (0, 1):
        for c in (0, 1):
            g = gy[:, a::2, c::2, :]
            gx += g @ w[a, c]
            gw[a, c] = g.reshape(-1, g.shape[3]).T @ x2
    return gx, gw, gy.sum(axis=(0, 1, 2))


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def param_shapes(levels=4, base=32, in_channels=3):
    """(name, shape) of every parameter tensor, in the flat order of the C interface."""
    C = [base << l for l in range(levels)]
    out = []
    cin = in_channels
    for l in range(levels):
        out += [(f"enc{l}a.w", (C[l], 3, 3, cin)), (f"enc{l}a.b", (C[l],)),
                (f"enc{l}b.w", (C[l], 3, 3, C[l])), (f"enc{l}b.b", (C[l],))]
        cin = C[l]
    for l in range(levels - 2, -1, -1):
        out += [(f"up{l}.w", (2, 2, C[l], C[l + 1])), (f"up{l}.b", (C[l],)),
                (f"dec{l}a.w", (C[l], 3, 3, 2 * C[l])), (f"dec{l}a.b", (C[l],)),
                (f"dec{l}b.w", (C[l], 3, 3, C[l])), (f"dec{l}b.b", (C[l],))]
    out += [("head.w", (C[0],)), ("head.b", (1,))]
    return out


def param_count(levels=4, base=32, in_channels=3):
    return int(sum(np.prod(s) for _, s in param_shapes(levels, base, in_channels)))


def unpack(theta, levels=4, base=32, in_channels=3):
    p, off = {}, 0
    for name, shp in param_shapes(levels, base, in_channels):
        k = int(np.prod(shp))
        p[name] = np.asarray(theta[off:off + k], dtype=np.float64).reshape(shp)
        off += k
    assert off == theta.size
    return p


def pack(p, levels=4, base=32, in_channels=3):
    return np.concatenate([p[name].reshape(-1) for name, _ in param_shapes(levels, base, in_channels)])


def init_params(rng, levels=4, base=32, in_channels=3):
    """He-normal weights and zero biases (drawn from rng; an input of the network)."""
    parts = []
    for name, shp in param_shapes(levels, base, in_channels):
        if name.endswith(".b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            fan_in = int(np.prod(shp[1:])) if not name.startswith("up") else shp[3]
            if name == "head.w":
                fan_in = shp[0]
            parts.append(rng.standard_normal(int(np.prod(shp))) * np.sqrt(2.0 / fan_in))
    return np.concatenate(parts)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
def forward(theta, x, levels=4, base=32, storage="fp64"):
    """x [n,H,W,Cin] -> y [n,H,W] and the activations the backward pass needs.

    storage="bf16": the input, the 3x3 and transposed-convolution weights and
    every stored activation are rounded to bfloat16 (see the module notes).
    """
    q = bf16 if storage == "bf16" else (lambda a: a)
    p = unpack(theta, levels, base, x.shape[3])
    for name in list(p):
        if name.endswith(".w") and name != "head.w":
            p[name] = q(p[name])
    x = q(x)
    cache = {"x": x, "p": p}
    h = x
    skips = []
    for l in range(levels):
        a = q(relu(conv3x3(h, p[f"enc{l}a.w"], p[f"enc{l}a.b"])))
        b = q(relu(conv3x3(a, p[f"enc{l}b.w"], p[f"enc{l}b.b"])))
        cache[f"enc{l}.in"], cache[f"enc{l}.a"], cache[f"enc{l}.b"] = h, a, b
        skips.append(b)
        if l < levels - 1:
            h, arg = maxpool2(b)
            cache[f"pool{l}.arg"] = arg
    h = skips[-1]
    for l in range(levels - 2, -1, -1):
        u = q(upconv2(h, p[f"up{l}.w"], p[f"up{l}.b"]))
        cat = np.concatenate([u, skips[l]], axis=3)
        a = q(relu(conv3x3(cat, p[f"dec{l}a.w"], p[f"dec{l}a.b"])))
        b = q(relu(conv3x3(a, p[f"dec{l}b.w"], p[f"dec{l}b.b"])))
        cache[f"up{l}.in"], cache[f"dec{l}.cat"], cache[f"dec{l}.a"], cache[f"dec{l}.b"] = h, cat, a, b
        h = b
    cache["head.in"] = h
    y = h @ p["head.w"] + p["head.b"][0]
    return y, cache


def backward(theta, cache, gy, levels=4, base=32):
    """Gradient of every parameter (flat, C-interface order) and of the input, given dL/dy."""
    x = cache["x"]
    p = cache["p"]   # the weights the forward pass used
    g = {}
    h = cache["head.in"]
    g["head.w"] = np.einsum("nhw,nhwc->c", gy, h)
    g["head.b"] = np.array([gy.sum()])
    gh = gy[..., None] * p["head.w"]
    gskip = {}
    # decoder levels in reverse forward order (level 0 feeds the head)
    for l in range(0, levels - 1):
        gb = gh * (cache[f"dec{l}.b"] > 0)
        ga, g[f"dec{l}b.w"], g[f"dec{l}b.b"] = conv3x3_bwd(cache[f"dec{l}.a"], p[f"dec{l}b.w"], gb)
        ga = ga * (cache[f"dec{l}.a"] > 0)
        gcat, g[f"dec{l}a.w"], g[f"dec{l}a.b"] = conv3x3_bwd(cache[f"dec{l}.cat"], p[f"dec{l}a.w"], ga)
        C = gcat.shape[3] // 2
        gu, gskip[l] = gcat[..., :C], gcat[..., C:]
        gh, g[f"up{l}.w"], g[f"up{l}.b"] = upconv2_bwd(cache[f"up{l}.in"], p[f"up{l}.w"], gu)
    # gh is now dL/d(encoder output of the deepest level)
    gx = None
    for l in range(levels - 1, -1, -1):
        gb = gh if l == levels - 1 else gskip[l] + gpool
        gb = gb * (cache[f"enc{l}.b"] > 0)
        ga, g[f"enc{l}b.w"], g[f"enc{l}b.b"] = conv3x3_bwd(cache[f"enc{l}.a"], p[f"enc{l}b.w"], gb)
        ga = ga * (cache[f"enc{l}.a"] > 0)
        gin, g[f"enc{l}a.w"], g[f"enc{l}a.b"] = conv3x3_bwd(cache[f"enc{l}.in"], p[f"enc{l}a.w"], ga)
        if l > 0:
            gpool = maxpool2_bwd(cache[f"enc{l - 1}.b"].shape, cache[f"pool{l - 1}.arg"], gin)
        else:
            gx = gin
    return pack(g, levels, base, x.shape[3]), gx


def loss_and_grad(theta, x, t, levels=4, base=32, storage="fp64"):
    y, cache = forward(theta, x, levels, base, storage)
    L, gy = mse(y, t)
    grad, _ = backward(theta, cache, gy, levels, base)
    return L, grad, y


def adam_step(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction (t counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    theta = theta - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return theta, m, v


# ---------------------------------------------------------------------------
# lattice <-> network fields
# ---------------------------------------------------------------------------
def encode(cls, solid_value, plane, phi0=None):
    """Input planes from a class field (low two bits nonzero = solid), and phi0 as a fourth if given."""
    s = (np.asarray(cls) & 3) != 0
    planes = [s.astype(np.float64), np.where(s, solid_value, 0.0), np.full(s.shape, float(plane))]
    if phi0 is not None:
        planes.append(np.asarray(phi0, dtype=np.float64))
    return np.stack(planes, axis=-1)


def target(rho, cls, rho_g, rho_l):
    s = (np.asarray(cls) & 3) != 0
    return np.where(s, 0.0, (np.asarray(rho, dtype=np.float64) - rho_g) / (rho_l - rho_g))


def smooth_fluid(phi, cls, r):
    """Mean of phi over the fluid nodes of each fluid node's (2r+1)^2 window,
    periodic images; 0 on solid nodes.  phi, cls: [ny][nx]."""
    phi = np.asarray(phi, dtype=np.float64)
    fl = (np.asarray(cls) & 3) == 0
    ny, nx = phi.shape
    out = np.zeros_like(phi)
    for y in range(ny):
        for x in range(nx):
            if not fl[y, x]:
                continue
            ys = [(y + d) % ny for d in range(-r, r + 1)]
            xs = [(x + d) % nx for d in range(-r, r + 1)]
            win = np.ix_(ys, xs)
            out[y, x] = phi[win][fl[win]].mean()
    return out


def warm_rho(phi, rho_ref, cls, rho_g, rho_l, cut=0.0, smooth=0):
    """Mass-exact density from phi on fluid nodes:
    rho_g + (rho_l - rho_g) s clamp((phi + delta - cut) / (1 - 2 cut), 0, 1),
    phi first replaced by smooth_fluid(phi, cls, smooth) when smooth > 0
    (phi, rho_ref, cls then [ny][nx]).

    delta solves sum_fluid clamp(...) = (M - n_f rho_g) / (rho_l - rho_g), M
    the fluid mass of rho_ref (found by scipy's brentq), and s = 1 up to the
    root finder's residual.
    """
    from scipy.optimize import brentq
    if smooth > 0:
        phi = smooth_fluid(phi, cls, smooth)
    fl = (np.asarray(cls) & 3) == 0
    ph = np.asarray(phi, dtype=np.float64)[fl]
    M = float(np.asarray(rho_ref, dtype=np.float64)[fl].sum())
    want = (M - fl.sum() * rho_g) / (rho_l - rho_g)
    g = lambda d: np.clip((ph + d - cut) / (1.0 - 2.0 * cut), 0.0, 1.0)
    delta = brentq(lambda d: g(d).sum() - want, -1.0, 1.0, xtol=1e-15, rtol=1e-15, maxiter=500)
    s = want / g(delta).sum()
    out = np.zeros(np.shape(cls))
    out[fl] = rho_g + (rho_l - rho_g) * s * g(delta)
    return out, M, delta


def forward_flops(H=256, W=256, levels=4, base=32, in_channels=3):
    """Multiply-add count x 2 of one forward pass of one sample (convolutions, transposed convolutions, head)."""
    C = [base << l for l in range(levels)]
    f = 0
    cin = in_channels
    for l in range(levels):
        P = (H >> l) * (W >> l)
        f += 2 * P * 9 * cin * C[l] + 2 * P * 9 * C[l] * C[l]
        cin = C[l]
    for l in range(levels - 2, -1, -1):
        P = (H >> l) * (W >> l)
        f += 2 * (P // 4) * C[l + 1] * 4 * C[l] + 2 * P * 9 * 2 * C[l] * C[l] + 2 * P * 9 * C[l] * C[l]
    f += 2 * H * W * C[0]
    return f
