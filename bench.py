"""Throughput of the multiphase LB step with in-step contact-angle measurement.

Workload (default): D3Q19 FP32, 256^3 walled box, sphere r=60 at (128,128,92),
drop r0=40 tangent on top, wall chemical potential 0.04 (the middle of the
paper's sweep), Tr=0.8, BGK tau=1, contact angle every 500 steps over 32
azimuthal sectors.  Inputs are synthetic and resident in HBM before timing.

Prints one JSON line: MLUPS (fluid-node updates per second), the roofline of
the dominant kernel (k_collide: per-kernel HIP-event timing on the stream it
runs on) and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes per launch of the dominant kernel from rocprofv3 counters: TCC_EA0_RDREQ_128B x 128 B +
# TCC_EA0_RDREQ_64B x 64 B read, TCC_EA0_WRREQ_64B x 64 B written (a plain 1 GiB copy reads as 8388608
# 128-byte and writes as 16777216 64-byte requests, exactly its bytes); valid only for the kernel as it
# stands when they were taken (profiles/k_step_d3q19_f32_256cube.md; the phase-field model's k_pf_collide in
# profiles/k_pf_collide_d3q19_f32_256cube.md, its writes that are not 64-byte requests counted as 32 bytes).
# Keyed by (kernel, lattice side, precision, collision, force model).
COUNTED_TRAFFIC = {("k_step", 256, "f32", "bgk", "chemical-potential"): 13015528 * 128 + 1550 * 64 + 21594750 * 64,
                   ("k_step", 256, "f32", "mrt", "chemical-potential"): 12774044 * 128 + 1700 * 64 + 21594828 * 64,
                   ("k_collide", 256, "f32", "bgk", "phase-field"):
                       24626936 * 128 + 2257 * 64 + 36426673 * 64 + 439204 * 32}
# the same for kb_collide of the batched solver on the seeded table, from FETCH_SIZE x 2 and WRITE_SIZE in KiB
# (the scaling of a plain copy; profiles/kb_collide_batch_d2q9_512cases.md), keyed by (number of cases,
# precision, force model)
BATCH_COUNTED_TRAFFIC = {(512, "f32", "chemical-potential"): (1392231 * 2 + 1386829) * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=256, help="lattice side (256 = the benchmark workload)")
    ap.add_argument("--precision", default="f32", choices=["f32", "f32mixed", "f64"])
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"])
    ap.add_argument("--mrt-rates", default="dhumieres", choices=["dhumieres", "paper2d"],
                    help="D3Q19 MRT rates: d'Humieres et al.'s set (s_e 1.19, s_eps 1.4, s_q 1.2, s_pi 1.4, "
                         "s_m 1.98), or the paper's D2Q9 rates carried over (1.64, 1.54, 1.9, 1.54, 1.9), which "
                         "blow this drop up")
    ap.add_argument("--step-kernel", default="auto", choices=["auto", "split"],
                    help="auto: the one-pass step where the lattice allows it; split: density pass + collision")
    ap.add_argument("--wall", default="halfway", choices=["halfway", "interpolated"],
                    help="curved-wall scheme of the sessile3d workload (interpolated: linear interpolated "
                         "bounce-back with the mass correction)")
    ap.add_argument("--model", default="chemical-potential", choices=["chemical-potential", "phase-field"],
                    help="force model of the sessile3d and batch workloads (the phase-field model runs the split "
                         "step, both population sets: 304 algorithmic bytes per fluid-node update in FP32 D3Q19, "
                         "144 in D2Q9)")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle steps at full size (0 = skip)")
    ap.add_argument("--cpu-steps-1t", type=int, default=1, help="oracle steps at full size on one thread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="sessile3d", choices=["sessile3d", "batch", "unet"],
                    help="sessile3d: the 256^3 D3Q19 benchmark; batch: 512 seeded D2Q9 cases in one batch; "
                         "unet: training steps of the warm-start U-Net at 256^2")
    ap.add_argument("--batch", type=int, default=32, help="unet: samples per training step")
    ap.add_argument("--cases", type=int, default=512)
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only time a plain device copy of GIB gibibytes (bandwidth / counter calibration)")
    return ap.parse_args()


def calibrate_copy(gib):
    """A plain copy kernel of known size: achieved GB/s and the bytes it must move."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * 4 * n
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "mean_ms": round(ms, 4),
                      "achieved_GBs": round(moved / (ms * 1e-3) / 1e9, 1)}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy > 0:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the step has no multi-GPU decomposition; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "unet":
        unet_bench(args)
        return
    import torch

    from paper_2202_06516_amd import lbm as G
    from paper_2202_06516_amd import workloads as W

    prec = {"f32": G.LBM_F32, "f32mixed": G.LBM_F32_MIXED, "f64": G.LBM_F64}[args.precision]
    elem = 8 if prec == G.LBM_F64 else 4
    wl = W.sessile_3d(mu_w=0.04, n=args.n)
    pf = args.model == "phase-field"
    extra = {}
    if pf:
        # the same geometry with the order parameter: phi_w = 0.04 on the sphere, Eq. 16 width 2 xi
        wl = dict(wl, model=2, W=W.PF_W)
        extra = dict(W.PF_PARAMS, model=G.LBM_MODEL_PHASE_FIELD)
    stream = torch.cuda.Stream()
    rates = {}
    if args.collision == "mrt":
        rates = (dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.4, s_m=1.98) if args.mrt_rates == "dhumieres"
                 else dict(s_e=1.64, s_eps=1.54, s_q=1.9, s_pi=1.54, s_m=1.9))
    lat = G.Lattice(G.LBM_D3Q19, n=wl["n"], precision=prec, axis_bc=(1, 1, 1), stream=stream.cuda_stream,
                    collision=G.LBM_BGK if args.collision == "bgk" else G.LBM_MRT,
                    bc_mode=G.LBM_BC_HALFWAY if args.wall == "halfway" else G.LBM_BC_BOUZIDI_MC,
                    tau=1.0, Tr=wl["Tr"], k=0.28, kappa=0.01,
                    step_kernel=G.LBM_STEP_AUTO if args.step_kernel == "auto" else G.LBM_STEP_SPLIT, **rates,
                    **extra)
    lat.set_solids(wl["solids"])
    lat.init_drops(wl["drops"], W=wl.get("W", 10.0))
    lat.set_measure(0, wl["n_sectors"])
    info = lat.info()
    n_fluid = info["n_fluid"]

    every = wl["every"]
    lat.step(args.warmup, measure_every=every)
    # untimed steps up to the next multiple of the cadence, so that the timed window starts with a
    # measured step whatever --steps and --warmup are
    align = (-args.warmup) % every
    if align:
        lat.step(align, measure_every=every)
    t_first = args.warmup + align
    n_measured = len(range(t_first, t_first + args.steps, every))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    series = lat.step(args.steps, measure_every=every, cap=n_measured)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat.sync()
    ms_step = dt * 1e3 / args.steps
    mlups = n_fluid * args.steps / dt / 1e6

    # cost of the in-step measurement: steps that all measure against steps that do not (not part of value)
    def per_step_ms(n, me):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(n, measure_every=me)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n
    n_ov = max(10, min(args.steps, 100))
    ms_meas, ms_plain = per_step_ms(n_ov, 1), per_step_ms(n_ov, 0)

    # per-kernel mean durations (HIP events around each launch on the context stream)
    prof = lat.profile(args.profile_steps)
    Q = 19
    # dominant kernel: the one-pass step k_step, or the split path's k_collide; algorithmic bytes per fluid
    # node = each population read once and written once (2 Q P; twice that with the phase-field model's
    # second population set)
    kern = "k_step" if "k_step" in prof else "k_collide"
    sets = 2 if pf else 1
    coll_bytes = n_fluid * 2 * Q * elem * sets
    coll_ms = prof[kern]
    achieved = coll_bytes / (coll_ms * 1e-3) / 1e9
    step_alg_bytes = 2 * Q * 4 * sets * n_fluid             # 152 B per fluid-node update (FP32), 304 phase field

    out = {
        "metric": "MLUPS (D3Q19 FP32 fluid-node updates/s) with %HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f32mixed": "f32 storage / f64 math", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"sessile drop on a sphere, D3Q19 {args.n}^3 walled box, sphere r={60 * args.n // 256}, "
                               f"drop r0={40 * args.n // 256}, mu_w=0.04, Tr={wl['Tr']}, {args.collision.upper()} tau=1, "
                               f"angle every {wl['every']} steps over {wl['n_sectors']} sectors"
                               + (", phase-field model (order parameter, wall phi_w=0.04)" if pf else "")
                               + (", interpolated wall" if args.wall == "interpolated" else ""),
                   "lattice": [args.n] * 3, "fluid_nodes": n_fluid, "precision": args.precision,
                   "collision": args.collision, **({"mrt_rates": rates} if rates else {})},
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # (counted in the default launch shape: none for another wall or plane chunk)
                     "traffic": (COUNTED_TRAFFIC.get((kern, args.n, args.precision, args.collision, args.model))
                                 if args.wall == "halfway" and "LBM_FUSED_ZC" not in os.environ else None),
                     "bytes_per_launch": coll_bytes, "mean_ms": round(coll_ms, 5)},
        "step_efficiency": {"algorithmic_bytes_per_update": 2 * Q * 4 * sets,
                            "achieved_GBs": round(step_alg_bytes / (ms_step * 1e-3) / 1e9, 1),
                            "frac_of_peak": round(step_alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms": {k: round(v, 5) for k, v in prof.items()},
        "angle": {"timed_window_steps": [t_first, t_first + args.steps], "measured_steps": n_measured,
                  "mean_deg": series[-1].mean_deg if series else None,
                  "n_valid": series[-1].n_valid if series else None,
                  "measured_step_overhead_ms": round(ms_meas - ms_plain, 5)},
    }
    if not args.no_cpu and args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps, args.collision, args.cpu_steps_1t)
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Aggregate throughput of the batched solver on the seeded case table."""
    import torch

    from paper_2202_06516_amd import lbm as G
    from paper_2202_06516_amd import workloads as W

    cases, acc = W.batch_cases(args.cases, seed=0)
    pf = args.model == "phase-field"
    extra = {}
    if pf:
        cases = W.pf_batch_cases(cases, seed=1)
        extra = dict(W.PF_PARAMS, model=G.LBM_MODEL_PHASE_FIELD)
    prec = {"f32": G.LBM_F32, "f32mixed": G.LBM_F32_MIXED, "f64": G.LBM_F64}[args.precision]
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    b = G.Batch(cases, precision=prec, autotune=True, stream=stream.cuda_stream, tau=1.0, Tr=0.8, k=0.28,
                kappa=0.01, collision=G.LBM_MRT, **extra)
    t_setup = time.perf_counter() - t0
    inf = b.info()
    b.step(args.warmup, measure_every=100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps, measure_every=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.sync()
    ang = b.angles()
    valid = sum(1 for a in ang if a.status == 0)
    # dominant kernel: kb_collide, timed with HIP events on the batch's stream over eager steps
    prof = b.profile(args.profile_steps)
    Q, P = 9, (8 if args.precision == "f64" else 4)
    # algorithmic: each population read once and written once (both sets of the phase-field model)
    coll_bytes = inf["fluid_nodes"] * 2 * Q * P * (2 if pf else 1)
    kern = "kb_pf_collide" if pf else "kb_collide"
    coll_ms = prof[kern]
    achieved = coll_bytes / (coll_ms * 1e-3) / 1e9
    what = ("R_s U[16,128], r0 U[12,96], mu_w U[-0.01,0.1], Tr=0.8, MRT tau=1, angle every 100" if not pf else
            "R_s U[16,128], r0 U[12,96], phase-field model, wall order parameter U[-0.4,0.4], MRT tau=1, "
            "angle every 100")
    out = {
        "metric": "aggregate MLUPS of the batched D2Q9 solver (fluid-node updates/s)",
        "value": round(inf["fluid_nodes"] * args.steps / dt / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4),
        "higher_is_better": True, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"{args.cases} seeded D2Q9 drop-on-cylinder cases (PCG64 seed 0), sides U[64,512], "
                               + what,
                   "total_nodes": inf["total_nodes"], "fluid_nodes": inf["fluid_nodes"], "accept_rate": acc,
                   "tile_w": inf["tile_w"], "blocks_per_cu": inf["blocks_per_cu"],
                   "tuned_ms_per_step": inf["tune_ms_per_step"], "setup_s": round(t_setup, 2)},
        "cases_with_contact_angle": valid,
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": BATCH_COUNTED_TRAFFIC.get((args.cases, args.precision, args.model)),
                     "bytes_per_launch": coll_bytes, "mean_ms": round(coll_ms, 5)},
        "kernels_ms": {k: round(v, 5) for k, v in prof.items()},
    }
    if not args.no_cpu and args.cpu_steps > 0:
        out["cpu_baseline"] = batch_cpu_baseline(cases[:16], 100, pf)
    print(json.dumps(out), flush=True)


def batch_cpu_baseline(cases, steps, pf=False):
    """The FP64 oracle on the first cases of the same seeded table, one lattice after another."""
    import oracle as O
    O.build(force=False)
    from paper_2202_06516_amd import workloads as W
    from tests.pairs import oracle_lattice
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fluid, dt = 0, 0.0
    for cs in cases:
        wl = dict(dim=2, n=cs["n"], wall=(0, 0), solids=[cs["solid"]], drops=[cs["drop"]])
        if pf:
            wl.update(model=2, W=W.PF_W)
        o = oracle_lattice(wl, Tr=0.8)
        t0 = time.perf_counter()
        o.step(steps)
        dt += time.perf_counter() - t0
        fluid += int((o.cls == 0).sum())
    return {"value": round(fluid * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of each of the first {len(cases)} cases (FP64 MRT, plain loops, OpenMP)"}


def unet_bench(args):
    """Training throughput of the warm-start U-Net (BF16 MFMA, FP32 accumulation) on synthetic inputs."""
    import numpy as np
    import torch

    from paper_2202_06516_amd import lbm as G
    from paper_2202_06516_amd import warmstart as WS

    B, H, W = args.batch, 256, 256
    stream = torch.cuda.Stream()
    net = G.Unet(H=H, W=W, batch=B, in_channels=WS.IN_CHANNELS, base_channels=32, levels=4,
                 stream=stream.cuda_stream)
    WS.init_params(net, seed=0)
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand((B, H, W, WS.IN_CHANNELS), device="cuda", generator=gen)
    t = torch.rand((B, H, W), device="cuda", generator=gen)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 200))
    warm = max(1, min(args.warmup, 50))
    for _ in range(warm):
        net.train_step(x.data_ptr(), t.data_ptr(), B)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        net.train_step(x.data_ptr(), t.data_ptr(), B)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    flops = 3 * WS.forward_flops(H, W) * B          # forward + data gradients + weight gradients
    tflops = flops / (ms * 1e-3) / 1e12
    out = {
        "metric": "U-Net training samples/s (256^2, 4 levels, 32..256 channels)", "value": round(B * steps / dt, 1),
        "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": round(dt * 1e3 / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)",
        "data": "synthetic",
        "config": {"workload": f"warm-start U-Net training step, batch {B}, 256x256, 4 inputs",
                   "params": net.n_params, "fwd_gflop_per_sample": round(WS.forward_flops(H, W) / 1e9, 3)},
        "roofline": {"bound": "mfma", "kernel": "whole training step, every kernel (HIP events on its stream)",
                     "achieved": round(tflops, 1), "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tflops / 2500.0, 4),
                     "traffic": None},
    }
    if not args.no_cpu:
        import oracle.unet_ref as U
        rng = np.random.default_rng(0)
        th = np.asarray(U.init_params(rng, 4, 32, WS.IN_CHANNELS))
        xs = rng.random((1, H, W, WS.IN_CHANNELS))
        ts = rng.random((1, H, W))
        c0 = time.perf_counter()
        U.loss_and_grad(th, xs, ts, 4, 32)
        cdt = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": round(1.0 / cdt, 4), "unit": "samples/s", "cores": os.cpu_count(),
                               "kind": "oracle", "sample": "one 256x256 sample, FP64 numpy forward + backward"}
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, steps, collision, steps_1t):
    """The FP64 oracle on the same lattice, timed over a few full-size steps with every OpenMP thread
    and over fewer steps on one thread."""
    import oracle as O
    O.build(force=False)
    from tests.pairs import oracle_lattice
    threads = O.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    o = oracle_lattice(wl, collision)
    n_fluid = int((o.cls == 0).sum())
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    out = {"value": round(n_fluid * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} steps of the full {wl['n'][0]}^3 lattice (FP64, plain loops, OpenMP)",
           "cpu_model": cpu_model()}
    if steps_1t > 0:
        O.set_threads(1)
        t0 = time.perf_counter()
        o.step(steps_1t)
        dt1 = time.perf_counter() - t0
        O.set_threads(threads)
        out["one_thread"] = {"value": round(n_fluid * steps_1t / dt1 / 1e6, 3), "unit": "MLUPS",
                             "sample": f"{steps_1t} more steps of the same lattice on one thread"}
    return out


if __name__ == "__main__":
    main()
