"""The BF16-MFMA U-Net (lbm_unet_*) against the FP64 oracle.

Forward outputs within 1e-2 of the float64 network and every parameter
tensor's gradient within 2e-2 (relative L2 norm; BF16 operands and
activations with FP32 accumulation), on shapes that are not multiples of
the tiles, and at the full 256 x 256 four-level size.  ReLU masks and
pooling choices are discrete decisions on forward values, so the gradients
are compared with the oracle run on bfloat16-stored forward values (its
arithmetic stays float64, its gradients unrounded); the forward output is
also compared with that run, more tightly.  Element by element as well: the
output no further from float64 than the oracle's own bfloat16-stored run (plus
a quarter), and every gradient element within 2e-2 of the largest of its
tensor (about 1e-2 at most on these shapes).  Gradients are deterministic;
one Adam step matches its definition applied to the library's own
gradients; training lowers the loss; the field kernels match their
definitions.
"""
import numpy as np
import pytest

from oracle import unet_ref as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def max_err(a, b):
    """Element-wise: max |a - b| over max |b|."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda")


def make_net(levels, base, H, W, batch, **kw):
    from paper_2202_06516_amd import lbm as G
    return G.Unet(H=H, W=W, batch=batch, base_channels=base, levels=levels, **kw)


def case(levels, base, H, W, n, seed):
    rng = np.random.default_rng(seed)
    th = U.init_params(rng, levels, base, 3)
    th += 0.02 * rng.standard_normal(th.size)
    th = th.astype(np.float32).astype(np.float64)
    x = rng.standard_normal((n, H, W, 3))
    t = rng.standard_normal((n, H, W))
    return th, x, t


def gpu_fwd_bwd(th, x, t, levels, base, batch=None):
    n, H, W, _ = x.shape
    net = make_net(levels, base, H, W, batch or n)
    assert net.n_params == th.size
    net.set_params(th)
    xd, td = dev(x), dev(t)
    yd = torch.empty((n, H, W), dtype=torch.float32, device="cuda")
    net.forward(xd.data_ptr(), yd.data_ptr(), n)
    loss = net.backward(xd.data_ptr(), td.data_ptr(), n)
    return yd.cpu().numpy().astype(np.float64), loss, net.grads().astype(np.float64), net


def check_against_oracle(levels, base, H, W, n, seed, batch=None, fwd_tol=1e-2, stored_tol=5e-3):
    th, x, t = case(levels, base, H, W, n, seed)
    y, loss, g, _ = gpu_fwd_bwd(th, x, t, levels, base, batch)
    y64, _ = U.forward(th, x, levels, base)
    L, g_ref, y_ref = U.loss_and_grad(th, x, t, levels, base, storage="bf16")
    print("forward vs fp64 %.2e (element-wise %.2e), vs bf16-stored %.2e (element-wise %.2e), "
          "oracle's own bf16 gap %.2e (element-wise %.2e)"
          % (rel(y, y64), max_err(y, y64), rel(y, y_ref), max_err(y, y_ref), rel(y_ref, y64), max_err(y_ref, y64)))
    assert rel(y, y64) <= fwd_tol, rel(y, y64)
    assert rel(y, y_ref) <= stored_tol, rel(y, y_ref)
    # element by element: no further from float64 than the oracle's own
    # bfloat16-stored run is (plus a quarter), and within twice the L2 bound of it
    assert max_err(y, y64) <= max(fwd_tol, 1.25 * max_err(y_ref, y64)), (max_err(y, y64), max_err(y_ref, y64))
    assert max_err(y, y_ref) <= 2 * stored_tol, max_err(y, y_ref)
    assert abs(loss - L) <= 1e-2 * L
    off = 0
    worst = []
    for name, shp in U.param_shapes(levels, base, 3):
        k = int(np.prod(shp))
        e = rel(g[off:off + k], g_ref[off:off + k])
        worst.append((e, name, max_err(g[off:off + k], g_ref[off:off + k])))
        off += k
    worst.sort(reverse=True)
    print("worst gradient errors (L2, name, element-wise):", worst[:4])
    print("largest element-wise gradient error:", max(worst, key=lambda w: w[2]))
    assert worst[0][0] <= 2e-2, worst[:4]
    assert max(w[2] for w in worst) <= 2e-2, max(worst, key=lambda w: w[2])


@pytest.mark.parametrize("levels,base,H,W,n", [
    (1, 8, 16, 16, 2),      # two convolutions and the head
    (2, 8, 12, 20, 3),      # pooling, transposed convolution, skip; 720 pixels: ragged tiles
    (3, 16, 32, 24, 2),
    (2, 32, 10, 6, 1),      # tiny: every tile ragged, level 1 is 5 x 3
    (2, 16, 6, 80, 2),      # rows of 80 and 40 pixels: ragged 128-, 64- and 32-pixel segments
])
def test_small_networks_match_the_oracle(levels, base, H, W, n):
    check_against_oracle(levels, base, H, W, n, seed=100 + levels * 10 + n)


def test_fewer_samples_than_the_batch():
    check_against_oracle(2, 16, 16, 16, 2, seed=7, batch=5)


def test_full_size_network_matches_the_oracle():
    # the warm-start network: 4 levels, 32..256 channels, 256 x 256.  Its 18
    # stored BF16 activations put the output about 1.1e-2 from float64 (the
    # oracle's own bfloat16-stored run shows the same gap): 2e-2 against
    # float64.  Against the bfloat16-stored oracle, sums accumulated in FP32
    # rather than float64 now and then round to the other neighbouring
    # bfloat16 value, and 18 layers carry that on: switching only the
    # oracle's accumulation to float32 moves its output by 7e-3 here, so
    # 1.5e-2 against the bfloat16-stored run
    check_against_oracle(4, 32, 256, 256, 1, seed=3, fwd_tol=2e-2, stored_tol=1.5e-2)


def test_gradients_are_deterministic():
    th, x, t = case(3, 16, 64, 64, 2, 11)
    _, l1, g1, net = gpu_fwd_bwd(th, x, t, 3, 16)
    xd, td = dev(x), dev(t)
    l2 = net.backward(xd.data_ptr(), td.data_ptr(), 2)
    g2 = net.grads()
    assert l1 == l2 and np.array_equal(g1.astype(np.float32), g2)


def test_adam_step_matches_its_definition():
    th, x, t = case(2, 16, 32, 32, 2, 12)
    net = make_net(2, 16, 32, 32, 2, lr=1e-3)
    net.set_params(th)
    xd, td = dev(x), dev(t)
    net.train_step(xd.data_ptr(), td.data_ptr(), 2)
    g = net.grads().astype(np.float64)
    w1 = net.params().astype(np.float64)
    ref, m, v = U.adam_step(th, np.zeros_like(th), np.zeros_like(th), g, 1, lr=1e-3)
    assert np.max(np.abs(w1 - ref)) <= 1e-6 * max(1.0, np.max(np.abs(th)))
    net.train_step(xd.data_ptr(), td.data_ptr(), 2)
    g2 = net.grads().astype(np.float64)
    w2 = net.params().astype(np.float64)
    ref2, _, _ = U.adam_step(ref, m, v, g2, 2, lr=1e-3)
    assert np.max(np.abs(w2 - ref2)) <= 2e-6 * max(1.0, np.max(np.abs(th)))


def test_training_lowers_the_loss():
    rng = np.random.default_rng(13)
    x = rng.standard_normal((4, 32, 32, 3))
    t = np.tanh(x[..., 0] - 0.5 * x[..., 1]) + 0.2 * x[..., 2]
    th = U.init_params(rng, 2, 16, 3)
    net = make_net(2, 16, 32, 32, 4, lr=2e-3)
    net.set_params(th)
    xd, td = dev(x), dev(t)
    losses = [net.train_step(xd.data_ptr(), td.data_ptr(), 4) for _ in range(150)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])


def test_bad_arguments_are_rejected():
    from paper_2202_06516_amd import lbm as G
    for kw in (dict(levels=0), dict(base_channels=12), dict(H=250, levels=4), dict(in_channels=9), dict(lr=-1.0)):
        with pytest.raises(G.LbmError):
            G.Unet(**{**dict(H=64, W=64, batch=2), **kw})
    net = make_net(2, 8, 16, 16, 2)
    x = dev(np.zeros((3, 16, 16, 3)))
    y = torch.empty((3, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(G.LbmError):
        net.forward(x.data_ptr(), y.data_ptr(), 3)       # more samples than the batch
    with pytest.raises(ValueError):
        net.set_params(np.zeros(5))


def test_field_kernels_match_their_definitions():
    from paper_2202_06516_amd import lbm as G
    rng = np.random.default_rng(21)
    n = 96 * 80
    cls = rng.choice(np.array([0, 0, 0, 4, 1, 2, 3], dtype=np.uint8), n)
    cd = dev(cls, torch.uint8)
    x = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    G.unet_encode(cd.data_ptr(), n, 0.4, 0.125, x.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), U.encode(cls, 0.4, 0.125).astype(np.float32))
    phi0 = rng.random(n).astype(np.float32)
    x4 = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    p0 = dev(phi0)
    G.unet_encode(cd.data_ptr(), n, -0.1, 0.5, x4.data_ptr(), phi0_ptr=p0.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(x4.cpu().numpy(), U.encode(cls, -0.1, 0.5, phi0).astype(np.float32))
    rho_g, rho_l = 0.0716, 6.43
    for prec, dt in ((G.LBM_F64, torch.float64), (G.LBM_F32, torch.float32)):
        rho = np.where(rng.random(n) < 0.3, rho_l, rho_g) * (1 + 0.01 * rng.standard_normal(n))
        rd = dev(rho, dt)
        phi = torch.empty(n, dtype=torch.float32, device="cuda")
        G.unet_target(rd.data_ptr(), prec, cd.data_ptr(), n, rho_g, rho_l, phi.data_ptr())
        torch.cuda.synchronize()
        ref = U.target(rd.cpu().numpy(), cls, rho_g, rho_l)
        assert np.allclose(phi.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
        # warm start from a blurred, shifted phi: exact mass, the oracle's density
        pred = np.clip(ref + 0.2 * rng.standard_normal(n) - 0.05, -0.3, 1.3).astype(np.float32)
        pd = dev(pred)
        out = torch.empty(n, dtype=dt, device="cuda")
        net = make_net(1, 8, 80, 96, 1)
        shape = (80, 96)
        for cut, smooth in ((0.0, 0), (0.1, 0), (0.05, 2)):
            info = net.warm_rho(pd.data_ptr(), rd.data_ptr(), cd.data_ptr(), 96, 80, prec, rho_g, rho_l,
                                out.data_ptr(), cut=cut, smooth=smooth)
            got = out.cpu().numpy().astype(np.float64)
            want, M, delta = U.warm_rho(pred.reshape(shape), rd.cpu().numpy().reshape(shape), cls.reshape(shape),
                                        rho_g, rho_l, cut=cut, smooth=smooth)
            want = want.reshape(-1)
            # the smoothed phi is an FP32 mean (about 1e-7 relative) on the GPU
            tol = (1e-12 if prec == G.LBM_F64 else 2e-7) if smooth == 0 else 1e-6
            assert abs(info["mass_ref"] - M) <= 1e-12 * M
            assert abs(got[(cls & 3) == 0].sum() - M) <= (1e-12 if prec == G.LBM_F64 else 2e-6) * M
            assert abs(info["delta"] - delta) <= (1e-9 if smooth == 0 else 1e-6)
            assert np.max(np.abs(got - want)) <= tol * rho_l * 4
            assert np.all(got[(cls & 3) != 0] == 0)
        with pytest.raises(G.LbmError):
            net.warm_rho(pd.data_ptr(), rd.data_ptr(), cd.data_ptr(), 96, 80, prec, rho_g, rho_l, out.data_ptr(),
                         cut=0.3)
        with pytest.raises(G.LbmError):      # smoothing needs nx ny <= H W of the network
            make_net(1, 8, 8, 8, 1).warm_rho(pd.data_ptr(), rd.data_ptr(), cd.data_ptr(), 96, 80, prec, rho_g,
                                             rho_l, out.data_ptr(), smooth=2)


def test_checkpoint_resumes_training_exactly(tmp_path):
    from paper_2202_06516_amd import lbm as G
    th, x, t = case(2, 16, 32, 32, 2, 14)
    xd, td = dev(x), dev(t)
    a = make_net(2, 16, 32, 32, 2)
    a.set_params(th)
    for _ in range(3):
        a.train_step(xd.data_ptr(), td.data_ptr(), 2)
    ck = tmp_path / "net.ckpt"
    a.save(ck)
    b = make_net(2, 16, 64, 48, 4)          # another lattice size and batch: same architecture
    b.load(ck)
    assert np.array_equal(a.params(), b.params())
    la = a.train_step(xd.data_ptr(), td.data_ptr(), 2)
    c = make_net(2, 16, 32, 32, 2)
    c.load(ck)
    lc = c.train_step(xd.data_ptr(), td.data_ptr(), 2)
    assert la == lc and np.array_equal(a.params(), c.params())   # Adam moments and step restored
    other = make_net(2, 8, 32, 32, 2)
    with pytest.raises(G.LbmError):
        other.load(ck)
    with pytest.raises(G.LbmError):
        a.load(tmp_path / "missing.ckpt")


def test_captured_training_steps_equal_eager_ones(monkeypatch):
    # the training step replays its forward and backward passes as graphs:
    # every replay (with eager launches and synchronisations in between, and a
    # new capture when the sample count changes) equals the eager step bit for bit
    th, x, t = case(3, 16, 64, 48, 3, 21)
    xd, td = dev(x), dev(t)
    g = make_net(3, 16, 64, 48, 3)
    monkeypatch.setenv("LBM_UNET_GRAPHS", "0")
    e = make_net(3, 16, 64, 48, 3)
    monkeypatch.delenv("LBM_UNET_GRAPHS")
    g.set_params(th)
    e.set_params(th)
    for n in (3, 3, 2, 3, 3):
        lg = g.train_step(xd.data_ptr(), td.data_ptr(), n)
        le = e.train_step(xd.data_ptr(), td.data_ptr(), n)
        torch.cuda.synchronize()
        assert lg == le, (n, lg, le)
        assert np.array_equal(g.params(), e.params()) and np.array_equal(g.grads(), e.grads()), n
