"""Pins of the FP64 U-Net oracle against definitions that do not come from it.

Each layer is checked against a library routine or brute force; the whole
backward pass against central finite differences of the loss; Adam against
its first-step closed form; the warm-start density against its defining
properties (exact mass, bounds, monotone in phi).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_ref as U


def test_conv3x3_equals_scipy_correlate_with_zero_padding():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 7, 5, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, i], w[o, :, :, i], mode="same", boundary="fill")
                             for i in range(3))
            assert np.allclose(y[n, :, :, o], ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_tap_convention_with_a_delta_kernel():
    # W[o, dy + 1, dx + 1, i] multiplies input pixel (h + dy, w + dx)
    x = np.arange(20.0).reshape(1, 4, 5, 1)
    w = np.zeros((1, 3, 3, 1))
    w[0, 2, 1, 0] = 1.0       # dy = +1, dx = 0
    y = U.conv3x3(x, w, np.zeros(1))[0, :, :, 0]
    assert np.array_equal(y[:3], x[0, 1:, :, 0]) and np.all(y[3] == 0)
    w[:] = 0
    w[0, 1, 0, 0] = 1.0       # dy = 0, dx = -1
    y = U.conv3x3(x, w, np.zeros(1))[0, :, :, 0]
    assert np.array_equal(y[:, 1:], x[0, :, :4, 0]) and np.all(y[:, 0] == 0)


def test_maxpool_against_brute_force_and_first_maximum_rule():
    rng = np.random.default_rng(2)
    x = rng.integers(0, 3, size=(2, 6, 4, 3)).astype(float)   # many ties
    y, arg = U.maxpool2(x)
    for n in range(2):
        for h in range(3):
            for w in range(2):
                for c in range(3):
                    win = [x[n, 2 * h, 2 * w, c], x[n, 2 * h, 2 * w + 1, c], x[n, 2 * h + 1, 2 * w, c],
                           x[n, 2 * h + 1, 2 * w + 1, c]]
                    assert y[n, h, w, c] == max(win)
                    assert arg[n, h, w, c] == win.index(max(win))
    gy = rng.standard_normal(y.shape)
    gx = U.maxpool2_bwd(x.shape, arg, gy)
    assert np.isclose(gx.sum(), gy.sum()) and np.count_nonzero(gx) <= gy.size


def test_upconv_against_loops_and_adjointness():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((2, 2, 6, 5))
    b = rng.standard_normal(6)
    y = U.upconv2(x, w, b)
    for n in range(2):
        for h in range(3):
            for ww in range(4):
                for a in range(2):
                    for c in range(2):
                        ref = b + w[a, c] @ x[n, h, ww]
                        assert np.allclose(y[n, 2 * h + a, 2 * ww + c], ref, rtol=1e-13)
    # <up(x), g> = <x, up^T(g)> and d<up(x), g>/dw = gw
    g = rng.standard_normal(y.shape)
    gx, gw, gb = U.upconv2_bwd(x, w, g)
    y0 = U.upconv2(x, w, np.zeros(6))
    assert np.isclose((y0 * g).sum(), (x * gx).sum(), rtol=1e-12)
    assert np.isclose((y0 * g).sum(), (w * gw).sum(), rtol=1e-12)
    assert np.allclose(gb, g.sum(axis=(0, 1, 2)))


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    g = rng.standard_normal((2, 5, 6, 4))
    y0 = U.conv3x3(x, w, np.zeros(4))
    gx, gw, gb = U.conv3x3_bwd(x, w, g)
    assert np.isclose((y0 * g).sum(), (x * gx).sum(), rtol=1e-12)
    assert np.isclose((y0 * g).sum(), (w * gw).sum(), rtol=1e-12)


@pytest.mark.parametrize("levels,base,H,W", [(1, 8, 6, 4), (2, 8, 8, 6), (3, 8, 8, 8), (4, 8, 16, 8)])
def test_gradients_match_central_differences(levels, base, H, W):
    rng = np.random.default_rng(10 + levels)
    th = U.init_params(rng, levels, base, 3)
    th += 0.01 * rng.standard_normal(th.size)   # nonzero biases
    x = rng.standard_normal((2, H, W, 3))
    t = rng.standard_normal((2, H, W))
    L, g, _ = U.loss_and_grad(th, x, t, levels, base)
    # along one tensor's unit direction the loss is piecewise quadratic (ReLU and
    # pooling are piecewise linear), so central differences are exact up to
    # rounding unless the step crosses a kink: a short step avoids them
    h = 1e-7
    for _ in range(4):
        v = rng.standard_normal(th.size)
        v /= np.linalg.norm(v)
        lp = U.mse(U.forward(th + h * v, x, levels, base)[0], t)[0]
        lm = U.mse(U.forward(th - h * v, x, levels, base)[0], t)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(1e-2, abs(fd))
    # every parameter tensor on its own (a dropped or misplaced term in one layer shows here)
    off = 0
    for name, shp in U.param_shapes(levels, base, 3):
        k = int(np.prod(shp))
        v = np.zeros(th.size)
        v[off:off + k] = rng.standard_normal(k)
        v /= np.linalg.norm(v)
        lp = U.mse(U.forward(th + h * v, x, levels, base)[0], t)[0]
        lm = U.mse(U.forward(th - h * v, x, levels, base)[0], t)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(1e-2, abs(fd)), name
        off += k


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    th = U.init_params(rng, 2, 8, 3)
    x = rng.standard_normal((1, 8, 8, 3))
    t = rng.standard_normal((1, 8, 8))
    y, cache = U.forward(th, x, 2, 8)
    _, gy = U.mse(y, t)
    _, gx = U.backward(th, cache, gy, 2, 8)
    v = rng.standard_normal(x.shape)
    h = 1e-6
    fd = (U.mse(U.forward(th, x + h * v, 2, 8)[0], t)[0] - U.mse(U.forward(th, x - h * v, 2, 8)[0], t)[0]) / (2 * h)
    assert abs(fd - (gx * v).sum()) <= 1e-6 * max(1.0, abs(fd))


def test_param_count_of_the_default_network():
    # 4 levels of 32/64/128/256 channels, 3 inputs (sum of the layer shapes written out by hand)
    enc = (32 * 27 + 32 + 32 * 288 + 32) + (64 * 288 + 64 + 64 * 576 + 64) + \
          (128 * 576 + 128 + 128 * 1152 + 128) + (256 * 1152 + 256 + 256 * 2304 + 256)
    dec = (4 * 128 * 256 + 128 + 128 * 9 * 256 + 128 + 128 * 9 * 128 + 128) + \
          (4 * 64 * 128 + 64 + 64 * 9 * 128 + 64 + 64 * 9 * 64 + 64) + \
          (4 * 32 * 64 + 32 + 32 * 9 * 64 + 32 + 32 * 9 * 32 + 32)
    assert U.param_count() == enc + dec + 33 == 1925601


def test_adam_first_step_closed_form():
    # with bias correction the first step is -lr g / (|g| + eps) for every weight
    rng = np.random.default_rng(6)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = U.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-2, eps=1e-8)
    assert np.allclose(new - th, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_mse_gradient_closed_form():
    y = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[1.0, 1.0], [1.0, 1.0]])
    L, g = U.mse(y, t)
    assert L == (0 + 1 + 4 + 16) / 4
    assert np.array_equal(g, 2 * (y - t) / 4)


def test_warm_rho_exact_mass_bounds_and_monotone():
    rng = np.random.default_rng(7)
    n = 40 * 30
    cls = np.zeros(n, dtype=np.uint8)
    cls[rng.random(n) < 0.2] = 1
    rho_g, rho_l = 0.05, 7.0
    ref = np.where(rng.random(n) < 0.3, rho_l, rho_g)
    phi = np.clip(rng.standard_normal(n) * 0.4 + 0.3, -0.2, 1.2)
    rho, M, delta = U.warm_rho(phi, ref, cls, rho_g, rho_l)
    fl = cls == 0
    assert np.isclose(rho[fl].sum(), M, rtol=1e-13)
    assert np.isclose(M, ref[fl].sum())
    assert np.all(rho[~fl] == 0)
    assert rho[fl].min() >= rho_g - 1e-12 and rho[fl].max() <= rho_l * (1 + 1e-9)
    order = np.argsort(phi[fl])
    assert np.all(np.diff(rho[fl][order]) >= -1e-12)
    # with a cut, predictions near 0 and 1 become exactly gas and liquid
    rho, M, delta = U.warm_rho(phi, ref, cls, rho_g, rho_l, cut=0.1)
    assert np.isclose(rho[fl].sum(), M, rtol=1e-13)
    lo = phi[fl] + delta <= 0.1
    hi = phi[fl] + delta >= 0.9
    assert lo.any() and hi.any()
    assert np.allclose(rho[fl][lo], rho_g, rtol=1e-12) and np.allclose(rho[fl][hi], rho[fl].max(), rtol=1e-12)
    assert np.all(np.diff(rho[fl][order]) >= -1e-12)


def test_encode_and_target_definitions():
    cls = np.array([0, 1, 2, 3, 4, 0], dtype=np.uint8)     # 4 = fluid with the boundary flag
    x = U.encode(cls, 0.5, 0.25)
    assert np.array_equal(x[:, 0], [0, 1, 1, 1, 0, 0])
    assert np.array_equal(x[:, 1], [0, 0.5, 0.5, 0.5, 0, 0])
    assert np.all(x[:, 2] == 0.25)
    x4 = U.encode(cls, 0.5, 0.25, phi0=np.arange(6) / 10)
    assert x4.shape == (6, 4) and np.array_equal(x4[:, :3], x) and np.array_equal(x4[:, 3], np.arange(6) / 10)
    rho = np.array([1.0, 9.0, 9.0, 9.0, 0.5, 3.0])
    t = U.target(rho, cls, 0.5, 3.0)
    assert np.allclose(t, [0.2, 0, 0, 0, 0.0, 1.0])


def test_bf16_rounding_equals_torch_cpu_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        # exact midpoints between neighbouring bfloat16 values, both parities
                        ((rng.integers(0x0080, 0x7F00, 2000).astype(np.uint32) << 16) + 0x8000)
                        .view(np.float32),
                        np.array([0.0, -0.0, 1.0, -3.5, 65504.0, 1e-30])]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(U.bf16(a), ref)


def test_bf16_storage_forward_stays_close_to_fp64():
    rng = np.random.default_rng(9)
    th = U.init_params(rng, 3, 8, 3)
    x = rng.standard_normal((2, 16, 16, 3))
    y64, _ = U.forward(th, x, 3, 8)
    y16, c = U.forward(th, x, 3, 8, storage="bf16")
    assert np.linalg.norm(y16 - y64) <= 2e-2 * np.linalg.norm(y64)
    for k, v in c.items():
        if isinstance(v, np.ndarray) and k.endswith((".a", ".b", ".cat")):
            assert np.array_equal(v, U.bf16(v)), k


def test_smoothing_definition():
    rng = np.random.default_rng(12)
    ny, nx = 9, 11
    cls = np.zeros((ny, nx), dtype=np.uint8)
    cls[3:6, 4:8] = 1                                  # a solid block
    const = np.full((ny, nx), 0.37)
    s = U.smooth_fluid(const, cls, 2)
    assert np.allclose(s[cls == 0], 0.37, rtol=0, atol=1e-15) and np.all(s[cls != 0] == 0)
    phi = rng.random((ny, nx))
    s = U.smooth_fluid(phi, cls, 1)
    # brute force at a node next to the block and at a node that wraps around the corner
    for (y, x) in ((2, 5), (0, 0)):
        vals = [phi[(y + dy) % ny, (x + dx) % nx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if cls[(y + dy) % ny, (x + dx) % nx] == 0]
        assert np.isclose(s[y, x], np.mean(vals), rtol=1e-14)
    # the window mean never leaves the range of the fluid values
    assert s[cls == 0].min() >= phi[cls == 0].min() and s[cls == 0].max() <= phi[cls == 0].max()
