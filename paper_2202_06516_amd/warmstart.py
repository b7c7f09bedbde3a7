"""Learned warm start of the multiphase lattice Boltzmann run.

The paper starts every drop from the profile of Eq. 16 (Sec. IV) and lets it
relax; this module replaces that start by the equilibrium predicted by the
U-Net of lbm_unet_* and measures what it saves.  Python only orders library
calls and reduces per-case angle series; every field operation runs in the
library's kernels:

1. ``generate``: the batched solver advances every case to (near)
   equilibrium; the inputs come from the CLASS field and the initial
   density (lbm_unet_encode, lbm_unet_target) and the target from the final
   density (lbm_unet_target), all on the device.
2. ``train``: Adam on the BF16 MFMA network (lbm_unet_train_step), seeded
   minibatch order, cosine learning-rate decay.
3. ``evaluate``: every test case runs twice in one batch, cold (Eq. 16) and
   warm (the network's phi smoothed over a 5 x 5 fluid window, made
   mass-exact by lbm_unet_warm_rho, predictions within ``cut`` of pure gas or
   liquid sent to it, and written with lbm_batch_write), both measured every
   ``every`` steps.  The steps to
   equilibrium of a run are the first measured step after which its angle
   stays within ``tol`` degrees of the cold run's final angle up to the
   horizon; a warm run that never settles there, or loses its contact line,
   counts as a fallback (one would rerun it cold).

Command line: ``python -m paper_2202_06516_amd.warmstart --help``.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbm as G
from . import workloads as WL

MU_SCALE = 10.0     # input channel 1: 10 mu_w on solid nodes
AREA_SCALE = 10.0   # input channel 2: 10 pi r0^2 / (H W) everywhere

SOLVER = dict(tau=1.0, Tr=0.8, k=0.28, kappa=0.01, collision=G.LBM_MRT)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the warm-start pipeline needs a GPU")
    return torch


def make_batch(cases, stream):
    return G.Batch(cases, precision=G.LBM_F32, autotune=False, tile_w=256, blocks_per_cu=8, stream=stream,
                   **SOLVER)


def plane_value(case):
    nx, ny = case["n"][0], case["n"][1]
    return AREA_SCALE * math.pi * case["drop"][1] ** 2 / (nx * ny)


IN_CHANNELS = 4     # solid, mu_w on the solid, drop area, phi of the cold initial state


def encode_cases(b, cases, x, first=0, stream=None):
    """Input planes of cases[i] (batch case first + i, still in its initial
    state) into x[i] (device [N,H,W,4])."""
    torch = _torch()
    H, W = cases[0]["n"][1], cases[0]["n"][0]
    inf = b.info()
    cls = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    rho = torch.empty((H, W), dtype=torch.float32, device="cuda")
    phi0 = torch.empty((H, W), dtype=torch.float32, device="cuda")
    for i, c in enumerate(cases):
        b.read_device(first + i, G.FIELD_CLASS, cls.data_ptr(), cls.numel())
        b.read_device(first + i, G.FIELD_RHO, rho.data_ptr(), rho.numel() * 4)
        G.unet_target(rho.data_ptr(), G.LBM_F32, cls.data_ptr(), H * W, inf["rho_g"], inf["rho_l"], phi0.data_ptr(),
                      stream)
        G.unet_encode(cls.data_ptr(), H * W, MU_SCALE * c["solid"]["mu_w"], plane_value(c), x[i].data_ptr(), stream,
                      phi0_ptr=phi0.data_ptr())
        torch.cuda.synchronize()


def generate(cases, steps, check_every=1000, stream=None, log=print):
    """Advance cases to equilibrium; returns inputs x, targets t (device) and per-case angles."""
    torch = _torch()
    H, W = cases[0]["n"][1], cases[0]["n"][0]
    t0 = time.perf_counter()
    b = make_batch(cases, stream)
    inf = b.info()
    rho_g, rho_l = inf["rho_g"], inf["rho_l"]
    n = len(cases)
    log(f"generate: {n} cases set up in {time.perf_counter() - t0:.1f} s")
    x = torch.empty((n, H, W, IN_CHANNELS), dtype=torch.float32, device="cuda")
    encode_cases(b, cases, x, stream=stream)
    hist = []
    t0 = time.perf_counter()
    for k in range(steps // check_every):
        b.step(check_every, measure_every=check_every)
        a = b.angles()
        hist.append([x.mean_deg if x.status == 0 else np.nan for x in a])
        if (k + 1) % 5 == 0:
            log(f"generate: {n} cases, step {(k + 1) * check_every}, {time.perf_counter() - t0:.1f} s")
    try:
        b.sync()
    except G.LbmError as e:   # a case that lost finiteness is left out of the data below
        if e.status != G.LBM_E_NONFINITE:
            raise
    seconds = time.perf_counter() - t0
    hist = np.array(hist)
    t = torch.empty((n, H, W), dtype=torch.float32, device="cuda")
    cls = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    keep = np.zeros(n, dtype=bool)
    for i in range(n):
        rho = b.read(i, G.FIELD_RHO)             # host copy: the finiteness check of the case
        keep[i] = bool(np.isfinite(rho).all()) and np.isfinite(hist[-1, i])
        b.read_device(i, G.FIELD_CLASS, cls.data_ptr(), cls.numel())
        rd = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).to("cuda")
        G.unet_target(rd.data_ptr(), G.LBM_F32, cls.data_ptr(), H * W, rho_g, rho_l, t[i].data_ptr(), stream)
        torch.cuda.synchronize()
    drift = np.abs(hist[-1] - hist[-2]) if len(hist) > 1 else np.full(n, np.nan)
    meta = dict(theta=hist[-1][keep], drift=drift[keep], converged=drift[keep] < 0.05, rho_g=rho_g, rho_l=rho_l,
                lups=float(inf["fluid_nodes"]) * steps, seconds=seconds, dropped=int(n - keep.sum()))
    b.close()
    if not keep.all():
        idx = torch.from_numpy(np.flatnonzero(keep)).to("cuda")
        x, t = x.index_select(0, idx).contiguous(), t.index_select(0, idx).contiguous()
    return x, t, meta


def init_params(net, seed):
    """He-normal weights (seeded numpy draws, the network's random input), zero biases."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    cfg = net.cfg
    C = [cfg.base_channels << l for l in range(cfg.levels)]
    parts = []

    def conv(co, ci):
        parts.append(rng.standard_normal(co * 9 * ci) * math.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))

    cin = cfg.in_channels
    for l in range(cfg.levels):
        conv(C[l], cin)
        conv(C[l], C[l])
        cin = C[l]
    for l in range(cfg.levels - 2, -1, -1):
        parts.append(rng.standard_normal(4 * C[l] * C[l + 1]) * math.sqrt(2.0 / C[l + 1]))
        parts.append(np.zeros(C[l]))
        conv(C[l], 2 * C[l])
        conv(C[l], C[l])
    parts.append(rng.standard_normal(C[0]) * math.sqrt(1.0 / C[0]))
    parts.append(np.zeros(1))
    theta = np.concatenate(parts).astype(np.float32)
    net.set_params(theta)
    return theta


def forward_flops(H, W, levels=4, base=32, in_channels=IN_CHANNELS):
    """2 x multiply-adds of one forward pass of one sample (3x3 and transposed convolutions, head)."""
    C = [base << l for l in range(levels)]
    f, cin = 0, in_channels
    for l in range(levels):
        P = (H >> l) * (W >> l)
        f += 2 * P * 9 * C[l] * (cin + C[l])
        cin = C[l]
    for l in range(levels - 2, -1, -1):
        P = (H >> l) * (W >> l)
        f += 2 * P * C[l + 1] * C[l] + 2 * P * 9 * C[l] * (2 * C[l] + C[l])
    return f + 2 * H * W * C[0]


def mean_loss(net, x, t):
    B = net.cfg.batch
    tot, n = 0.0, x.shape[0]
    for i in range(0, n, B):
        m = min(B, n - i)
        tot += net.loss(x[i].data_ptr(), t[i].data_ptr(), m) * m
    return tot / n


def train(net, x, t, epochs, lr=1e-3, seed=0, xv=None, tv=None, log=print, stream=None):
    """Adam over seeded minibatch permutations with cosine decay; returns the loss history."""
    torch = _torch()
    B = net.cfg.batch
    n = x.shape[0]
    per_epoch = n // B
    total = max(1, epochs * per_epoch)
    rng = np.random.default_rng(np.random.PCG64(seed))
    hist = []
    step = 0
    t0 = time.perf_counter()
    for e in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to("cuda")
        run = 0.0
        for i in range(per_epoch):
            idx = perm[i * B:(i + 1) * B]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            torch.cuda.synchronize()
            net.set_lr(lr * 0.5 * (1.0 + math.cos(math.pi * step / total)) + 1e-6)
            run += net.train_step(xb.data_ptr(), tb.data_ptr(), B)
            step += 1
        rec = dict(epoch=e + 1, train=run / max(1, per_epoch), seconds=time.perf_counter() - t0)
        if xv is not None:
            rec["val"] = mean_loss(net, xv, tv)
        hist.append(rec)
        if (e + 1) % max(1, epochs // 10) == 0 or e == epochs - 1:
            log("train: " + json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in rec.items()}))
    return hist


def settle_step(series, ref, tol, every):
    """First measured step after which |theta - ref| <= tol up to the end (None if never)."""
    ok = np.isfinite(series) & (np.abs(series - ref) <= tol)
    if not ok[-1]:
        return None
    k = len(ok) - 1
    while k > 0 and ok[k - 1]:
        k -= 1
    return (k + 1) * every


def evaluate(net, cases, horizon, every=100, tol=0.5, cut=0.05, smooth=2, stream=None, log=print):
    """Cold vs warm steps to equilibrium of the test cases (both in one batch)."""
    torch = _torch()
    n = len(cases)
    H, W = cases[0]["n"][1], cases[0]["n"][0]
    b = make_batch(cases + cases, stream)
    inf = b.info()
    rho_g, rho_l = inf["rho_g"], inf["rho_l"]
    x = torch.empty((n, H, W, IN_CHANNELS), dtype=torch.float32, device="cuda")
    encode_cases(b, cases, x, first=n, stream=stream)
    phi = torch.empty((n, H, W), dtype=torch.float32, device="cuda")
    B = net.cfg.batch
    for i in range(0, n, B):
        net.forward(x[i].data_ptr(), phi[i].data_ptr(), min(B, n - i))
    rho_ref = torch.empty((H, W), dtype=torch.float32, device="cuda")
    cls = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    rho_new = torch.empty((H, W), dtype=torch.float32, device="cuda")
    mass_err = 0.0
    for i in range(n):
        b.read_device(n + i, G.FIELD_RHO, rho_ref.data_ptr(), rho_ref.numel() * 4)
        b.read_device(n + i, G.FIELD_CLASS, cls.data_ptr(), cls.numel())
        info = net.warm_rho(phi[i].data_ptr(), rho_ref.data_ptr(), cls.data_ptr(), W, H, G.LBM_F32, rho_g, rho_l,
                            rho_new.data_ptr(), cut=cut, smooth=smooth)
        mass_err = max(mass_err, abs(info["mass_written"] - info["mass_ref"]) / info["mass_ref"])
        b.write_rho_device(n + i, rho_new.data_ptr(), rho_new.numel() * 4)
    series = np.full((horizon // every, 2 * n), np.nan)
    t0 = time.perf_counter()
    for k in range(horizon // every):
        b.step(every, measure_every=every)
        a = b.angles()
        series[k] = [y.mean_deg if y.status == 0 else np.nan for y in a]
        if (k + 1) % max(1, (horizon // every) // 10) == 0:
            log(f"evaluate: step {(k + 1) * every}, {time.perf_counter() - t0:.1f} s")
    nonfinite = False
    try:
        b.sync()
    except G.LbmError as e:      # a run that lost finiteness keeps NaN angles: a fallback
        if e.status != G.LBM_E_NONFINITE:
            raise
        nonfinite = True
    b.close()
    cold, warm = series[:, :n], series[:, n:]
    ref = cold[-1]
    # the cold run must itself have settled: within tol/5 over the last 10 samples
    tail = max(1, min(10, len(cold) - 1))
    settled = np.isfinite(ref) & (np.nanmax(np.abs(cold[-tail - 1:] - ref), axis=0) <= tol / 5)
    res = []
    for i in range(n):
        sc = settle_step(cold[:, i], ref[i], tol, every)
        sw = settle_step(warm[:, i], ref[i], tol, every)
        late = warm[len(warm) // 2:, i]
        res.append(dict(case=i, theta_ref=float(ref[i]), cold=sc, warm=sw, settled=bool(settled[i]),
                        theta_warm0=float(warm[0, i]), theta_cold0=float(cold[0, i]),
                        theta_warm_end=float(warm[-1, i]),
                        warm_late_maxdev=float(np.nanmax(np.abs(late - ref[i]))) if np.isfinite(late).any() else None))
    use = [r for r in res if r["settled"] and r["cold"] is not None]
    ok = [r for r in use if r["warm"] is not None]
    ratios = np.array([r["cold"] / r["warm"] for r in ok]) if ok else np.array([np.nan])
    summary = dict(cases=n, evaluated=len(use), fallbacks=len(use) - len(ok),
                   median_cold=float(np.median([r["cold"] for r in use])) if use else None,
                   median_warm=float(np.median([r["warm"] for r in ok])) if ok else None,
                   median_ratio=float(np.median(ratios)), mean_ratio=float(np.mean(ratios)),
                   max_rel_mass_error=mass_err, tol_deg=tol, every=every, horizon=horizon, cut=cut, smooth=smooth,
                   any_nonfinite=nonfinite)
    return summary, res, series


def run(train_cases, val_cases, test_cases, gen_steps, horizon, epochs, levels=4, base=32, batch=8, lr=1e-3,
        seed=0, log=print, ckpt=None, cut=0.05, smooth=2, resume=None):
    """The whole pipeline on one GPU; returns a JSON-able report.  With resume,
    training continues from that checkpoint (weights, Adam moments and step) on
    the new cases, so that a larger training set can be seen chunk by chunk."""
    torch = _torch()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        rep = {}
        x, t, meta = generate(train_cases, gen_steps, stream=st.cuda_stream, log=log)
        rep["train_data"] = dict(cases=len(train_cases), dropped=meta["dropped"],
                                 converged=int(meta["converged"].sum()),
                                 seconds=round(meta["seconds"], 2),
                                 glups=round(meta["lups"] / meta["seconds"] / 1e9, 2))
        xv = tv = None
        if val_cases:
            xv, tv, mv = generate(val_cases, gen_steps, stream=st.cuda_stream, log=log)
        H, W = train_cases[0]["n"][1], train_cases[0]["n"][0]
        net = G.Unet(H=H, W=W, batch=batch, in_channels=IN_CHANNELS, base_channels=base, levels=levels, lr=lr,
                     stream=st.cuda_stream)
        if resume:
            net.load(resume)
        else:
            init_params(net, seed)
        t0 = time.perf_counter()
        hist = train(net, x, t, epochs, lr=lr, seed=seed + 1, xv=xv, tv=tv, log=log)
        rep["training"] = dict(epochs=epochs, seconds=round(time.perf_counter() - t0, 2), params=net.n_params,
                               first=hist[0], last=hist[-1])
        if ckpt:
            net.save(ckpt)
        del x, t
        summary, res, _ = evaluate(net, test_cases, horizon, cut=cut, smooth=smooth, stream=st.cuda_stream, log=log)
        rep["warm_start"] = summary
        rep["cases"] = res
        net.close()
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned warm start: data, training, cold vs warm evaluation")
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--train", type=int, default=1024)
    ap.add_argument("--val", type=int, default=64)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--gen-steps", type=int, default=40000)
    ap.add_argument("--horizon", type=int, default=40000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--ckpt", default=None, help="write the trained network here (or read it with --eval-only)")
    ap.add_argument("--eval-only", action="store_true", help="load --ckpt and only run the cold/warm evaluation")
    ap.add_argument("--resume", default=None, help="continue training from this checkpoint on the new cases")
    ap.add_argument("--train-seed", type=int, default=WL.WARM_SEEDS["train"],
                    help="seed of the training cases (a chunk of a larger set: a seed below the validation one)")
    ap.add_argument("--cut", type=float, default=0.05)
    ap.add_argument("--smooth", type=int, default=2, help="radius of the fluid-window mean applied to predictions")
    a = ap.parse_args(argv)
    kw = dict(side=a.side)
    if a.side != 256:   # radii scale with the lattice
        s = a.side / 256.0
        kw.update(rs=(max(12.0, 16.0 * s), 64.0 * s), r0=(max(18.0, 18.0 * s), max(20.0, 48.0 * s)))
    te = WL.warmstart_cases(a.test, WL.WARM_SEEDS["test"], **kw)
    log = lambda s: print(s, flush=True)
    if a.eval_only:
        torch = _torch()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            net = G.Unet(H=a.side, W=a.side, batch=8, in_channels=IN_CHANNELS, base_channels=a.base,
                         levels=a.levels, stream=st.cuda_stream)
            net.load(a.ckpt)
            summary, res, _ = evaluate(net, te, a.horizon, cut=a.cut, smooth=a.smooth, stream=st.cuda_stream, log=log)
        rep = dict(warm_start=summary, cases=res)
    else:
        if not a.train_seed < WL.WARM_SEEDS["val"]:
            ap.error("--train-seed must stay below the validation and test seeds")
        tr = WL.warmstart_cases(a.train, a.train_seed, **kw)
        va = WL.warmstart_cases(a.val, WL.WARM_SEEDS["val"], **kw) if a.val else []
        rep = run(tr, va, te, a.gen_steps, a.horizon, a.epochs, levels=a.levels, base=a.base, lr=a.lr, log=log,
                  ckpt=a.ckpt, cut=a.cut, smooth=a.smooth, resume=a.resume)
    line = json.dumps({k: v for k, v in rep.items() if k != "cases"})
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1, default=float)
    return 0


if __name__ == "__main__":
    sys.exit(main())
