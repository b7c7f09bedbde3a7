"""Parameter sweeps of Sec. IV A-B on the batched solver.

Every sweep is a set of independent 2-D cases -- a drop on a circular bump of
radius R rising H above a walled floor (Fig. 2a) -- advanced together by the
batched solver until every measured angle has settled, then reduced to the
statistics the paper reports:

- ``wettability``: theta against mu_w (Fig. 3) and the relative L2 deviation
  of theta(mu_w) from its least-squares line (the error E of Sec. IV A, its
  integrals taken as sums over the sampled mu_w);
- ``size``: theta for drop radii r0 = 30..100 on each of five wettabilities
  (Fig. 4a) and its standard deviation over r0;
- ``curvature``: theta for bump radii R = 150..400 (Fig. 4b) and its standard
  deviation over R;
- ``gravity``: sessile drops of growing radius under gravity (Sec. IV C,
  Fig. 5-6), or with the gravity reversed pendent ones (Fig. 7-8): the
  measured angle against the spherical-cap angle as the drops deform, and
  the radii at which a pendent drop detaches;
- ``sc-wettability``: the same measurement on the pseudopotential model
  (Sec. V), theta against the wall density on single lattices;
- ``pf-wettability``: on the phase-field model (Sec. V), theta against the
  wall order parameter on single lattices;
- ``sessile3d``: the 256^3 sessile drop of the benchmark workload (D3Q19 FP32,
  one-pass step) for several wall chemical potentials, its 32-sector measured
  angle against the apparent angle of a sphere fitted to the drop (the 3-D
  counterpart of the spherical-cap check of Sec. IV A), with either wall.

Each case also gets the spherical-cap angle of Sec. IV A from its final
density (base length L between the two measured contact points, cap height
above that chord, theta = beta - alpha on the convex bump).  Python orders
library calls and reduces angle series and one density read per case; every
step of the method runs in the library's kernels.

Command line: ``python -m paper_2202_06516_amd.sweeps --help``.
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


def make_batch(cases, Tr, precision=G.LBM_F32, stream=None, k=0.28, kappa=0.01, g=0.0, g_start=0,
               bc_mode=G.LBM_BC_HALFWAY):
    # the floor and ceiling are two solid layers (walled along y), x periodic;
    # g > 0 pulls toward the floor (sessile), g < 0 away from it (pendent)
    return G.Batch(cases, precision=precision, axis_bc=(0, 1, 0), tile_w=256, blocks_per_cu=8, stream=stream,
                   tau=1.0, Tr=Tr, k=k, kappa=kappa, collision=G.LBM_MRT, g=(0.0, -g, 0.0), g_start_step=g_start,
                   bc_mode=bc_mode)


def settle(b, every=1000, tol=0.02, min_steps=10000, max_steps=200000, log=print):
    """Step until every valid case's angle moved by less than tol degrees over
    the last interval (after min_steps), or max_steps.  Returns the angle
    history [intervals, cases] (NaN where a case had no contact line)."""
    hist = []
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        b.step(every, measure_every=every)
        steps += every
        hist.append([a.mean_deg if a.status == 0 else math.nan for a in b.angles()])
        if len(hist) >= 2 and steps >= min_steps:
            d = np.abs(np.array(hist[-1]) - np.array(hist[-2]))
            if np.all(d[np.isfinite(d)] < tol):
                break
        if steps % (10 * every) == 0:
            log(f"sweep: step {steps}, {time.perf_counter() - t0:.1f} s")
    try:
        b.sync()
    except G.LbmError as e:   # a case that lost finiteness keeps NaN below
        if e.status != G.LBM_E_NONFINITE:
            raise
    return np.array(hist), steps, time.perf_counter() - t0


def cap_angle(rho, cls, rho_m, centre, R, contact):
    """Spherical-cap angle (Sec. IV A) of a drop on a convex circle: base L
    between the two contact points, height Hc of the interface above that chord,
    R0 = (4 Hc^2 + L^2) / 8 Hc, tan beta = L / 2 (R0 - Hc), theta = beta - alpha
    with alpha = asin(L / 2R) the chord's half-angle seen from the centre."""
    ny, nx = rho.shape
    fl = cls == 0
    pts = []
    for dx, dy in ((1, 0), (0, 1)):
        r0, r1 = rho[: ny - dy, : nx - dx], rho[dy:, dx:]
        ok = fl[: ny - dy, : nx - dx] & fl[dy:, dx:] & ((r0 - rho_m) * (r1 - rho_m) < 0)
        yy, xx = np.nonzero(ok)
        t = (rho_m - r0[ok]) / (r1[ok] - r0[ok])
        pts.append(np.c_[xx + t * dx, yy + t * dy])
    pts = np.vstack(pts)
    c1, c2 = np.asarray(contact[0][:2]), np.asarray(contact[1][:2])
    L = float(np.linalg.norm(c2 - c1))
    mid = 0.5 * (c1 + c2)
    up = mid - np.asarray(centre[:2])
    up /= np.linalg.norm(up)
    Hc = float(np.max((pts - mid) @ up))
    if not (L > 0 and Hc > 0 and L < 2 * R):
        return math.nan
    R0 = (4 * Hc * Hc + L * L) / (8 * Hc)
    beta = math.degrees(math.atan2(L, 2 * (R0 - Hc)))
    return beta - math.degrees(math.asin(0.5 * L / R))


def linear_fit_error(x, y):
    """Least-squares line F through (x, y) and E = ||y - F|| / ||F||."""
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    A = np.c_[x, np.ones_like(x)]
    (a, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    F = a * x + c
    return float(np.linalg.norm(y - F) / np.linalg.norm(F)), float(a), float(c)


def run(kind, Tr=0.6, precision=G.LBM_F32, scale=1.0, mu=None, values=None, every=1000, tol=0.02,
        min_steps=10000, max_steps=200000, k=0.28, kappa=0.01, g=0.0, g_start=0, stream=None, log=print,
        bc_mode=G.LBM_BC_HALFWAY):
    cases, labels = WL.sweep_cases(kind, scale=scale, mu=mu, values=values)
    nx, ny = cases[0]["n"]
    H = 100.0 * scale
    b = make_batch(cases, Tr, precision, stream, k=k, kappa=kappa, g=g, g_start=g_start, bc_mode=bc_mode)
    min_steps = max(min_steps, g_start + 2 * every)
    inf = b.info()
    rho_m = 0.5 * (inf["rho_g"] + inf["rho_l"])
    log(f"sweep {kind}: {len(cases)} cases of {nx}x{ny}, Tr = {Tr}")
    hist, steps, seconds = settle(b, every, tol, min_steps, max_steps, log)
    final = b.angles()
    res = []
    for i, (cs, (v, m)) in enumerate(zip(cases, labels)):
        th = hist[-1, i]
        drift = float(abs(hist[-1, i] - hist[-2, i])) if len(hist) > 1 else math.nan
        cap = math.nan
        if math.isfinite(th):
            rho = b.read(i, G.FIELD_RHO)[0].astype(np.float64)
            cls = b.read(i, G.FIELD_CLASS)[0]
            if np.isfinite(rho).all():
                cap = cap_angle(rho, cls, rho_m, cs["solid"]["center"], cs["solid"]["radius"], final[i].contact)
        res.append(dict(value=float(v), mu_w=float(m), theta=float(th), cap=float(cap), drift=drift,
                        sectors=[float(final[i].sector_deg[k]) for k in range(2)],
                        contact=[[round(float(final[i].contact[k][d]), 2) for d in range(2)] for k in range(2)]))
    b.close()
    out = dict(kind=kind, Tr=Tr, k=k, kappa=kappa, g=g, g_start=g_start, nx=nx, ny=ny, H=H,
               wall="interpolated" if bc_mode == G.LBM_BC_BOUZIDI_MC else "halfway", steps=steps, seconds=round(seconds, 2),
               mlups=round(float(inf["fluid_nodes"]) * steps / seconds / 1e6, 1), cases=res)
    ok = [r for r in res if math.isfinite(r["theta"])]
    if kind == "wettability" and len(ok) >= 3:
        E, a, c = linear_fit_error([r["mu_w"] for r in ok], [r["theta"] for r in ok])
        out.update(E=round(E, 4), slope_deg_per_mu=round(a, 2), intercept_deg=round(c, 2))
        okc = [r for r in ok if math.isfinite(r["cap"])]
        if okc:
            out["max_abs_theta_minus_cap"] = round(max(abs(r["theta"] - r["cap"]) for r in okc), 2)
    if kind == "gravity":
        # Sec. IV C: the drops flatten as r0 grows, so the spherical-cap angle
        # drifts while the microscopic angle should not
        per = {}
        for r in res:
            per.setdefault(r["mu_w"], []).append(r)
        out["per_mu"] = {}
        for m, rs in sorted(per.items()):
            ok_ = [r for r in rs if math.isfinite(r["theta"])]
            th = np.array([r["theta"] for r in ok_])
            cp = np.array([r["cap"] for r in ok_])
            out["per_mu"][str(m)] = dict(
                r0=[r["value"] for r in ok_], theta=[round(float(v), 2) for v in th], cap=[round(float(v), 2) for v in cp],
                theta_std=round(float(th.std()), 3) if len(th) else None,
                cap_change=round(float(cp[-1] - cp[0]), 2) if len(cp) > 1 else None,
                detached=[r["value"] for r in rs if not math.isfinite(r["theta"])])
    if kind in ("size", "curvature"):
        per = {}
        for r in ok:
            per.setdefault(r["mu_w"], []).append(r["theta"])
        out["per_mu"] = {str(m): dict(mean=round(float(np.mean(t)), 2), std=round(float(np.std(t)), 3), n=len(t))
                         for m, t in sorted(per.items())}
    out["invalid"] = len(res) - len(ok)
    return out


def _lattice_wettability(kind, make, values, read_field, rho_m, n, R, r0, steps, every, W, log):
    """Drops on a cylinder of radius R in a periodic n x n lattice, one lattice
    per wall value (made by make(value)), each run to steps: the measured angle
    and the spherical-cap angle of the final drop (isolevel rho_m of the field
    read_field(lattice) returns)."""
    res = []
    t0 = time.perf_counter()
    for v in values:
        lat = make(v)
        c = (n / 2.0, 10.0 + R)
        lat.set_solids([dict(center=c, radius=R, mu_w=v)])
        lat.init_drops([((c[0], c[1] + R + r0), r0)], W=W)
        lat.set_measure(0, 2)
        ser = lat.step(steps, measure_every=every, cap=steps // every + 1)
        a = ser[-1]
        th = a.mean_deg if a.status == 0 else math.nan
        drift = abs(ser[-1].mean_deg - ser[-2].mean_deg) if len(ser) > 1 and a.status == 0 else math.nan
        cap = math.nan
        if math.isfinite(th):
            fld = read_field(lat)[0].astype(np.float64)
            cls = lat.read(G.FIELD_CLASS)[0]
            cap = cap_angle(fld, cls, rho_m, c, R, a.contact)
        lat.close()
        res.append(dict(wall=v, theta=float(th), cap=float(cap), drift=float(drift),
                        sectors=[float(a.sector_deg[0]), float(a.sector_deg[1])]))
        log(f"{kind}: wall value {v}: theta {th:.2f}, cap {cap:.2f}, {time.perf_counter() - t0:.1f} s")
    ok = [r for r in res if math.isfinite(r["theta"])]
    out = dict(kind=kind, n=n, R=R, r0=r0, steps=steps, cases=res)
    d = [abs(r["theta"] - r["cap"]) for r in ok if math.isfinite(r["cap"])]
    if d:
        out.update(max_abs_theta_minus_cap=round(max(d), 2), mean_abs_theta_minus_cap=round(float(np.mean(d)), 2))
    return out


def sc_wettability(rho_w=(0.3, 0.5, 0.7, 0.9, 1.1, 1.3, 1.5), n=256, R=48.0, r0=36.0, steps=40000, every=1000,
                   precision=G.LBM_F64, log=print):
    """The measurement on the pseudopotential model (Sec. V): theta and the
    cap angle against the wall density rho_w.  The cases run one after the
    other on single lattices."""
    def make(v):
        return G.Lattice(G.LBM_D2Q9, n=(n, n, 1), precision=precision, tau=1.0, collision=G.LBM_MRT,
                         model=G.LBM_MODEL_PSEUDOPOTENTIAL, sc_G=WL.SC_G, rho_l=WL.SC_RHO_L, rho_g=WL.SC_RHO_G)
    out = _lattice_wettability("sc-wettability", make, rho_w, lambda lat: lat.rho, 0.5 * (WL.SC_RHO_L + WL.SC_RHO_G),
                               n, R, r0, steps, every, 5.0, log)
    out["G"] = WL.SC_G
    return out


def pf_wettability(phi_w=(-0.6, -0.4, -0.2, 0.0, 0.2, 0.4, 0.6), n=256, R=48.0, r0=36.0, steps=40000, every=1000,
                   precision=G.LBM_F64, log=print):
    """The measurement on the phase-field model (Sec. V): theta and the cap
    angle against the wall order parameter phi_w, read on phi at the isolevel 0."""
    def make(v):
        return G.Lattice(G.LBM_D2Q9, n=(n, n, 1), precision=precision, tau=1.0, collision=G.LBM_MRT,
                         model=G.LBM_MODEL_PHASE_FIELD, **WL.PF_PARAMS)
    out = _lattice_wettability("pf-wettability", make, phi_w, lambda lat: lat.phi, 0.0, n, R, r0, steps, every,
                               WL.PF_W, log)
    out.update(WL.PF_PARAMS)
    return out


def sessile3d(mu_w=(-0.01, 0.04, 0.1), n=256, steps=20000, every=1000, wall="halfway", log=print):
    """The benchmark's sessile layout per wall chemical potential: the mean of
    the 32 sector angles at the end, its spread over the sectors, the drift over
    the last interval, and the apparent angle of the final drop."""
    from .striped import apparent_angle
    res = []
    t0 = time.perf_counter()
    for m in mu_w:
        wl = WL.sessile_3d(mu_w=m, n=n)
        lat = G.Lattice(G.LBM_D3Q19, n=wl["n"], precision=G.LBM_F32, axis_bc=(1, 1, 1), collision=G.LBM_BGK,
                        bc_mode=G.LBM_BC_BOUZIDI_MC if wall == "interpolated" else G.LBM_BC_HALFWAY, tau=1.0,
                        Tr=wl["Tr"], k=0.28, kappa=0.01)
        lat.set_solids(wl["solids"])
        lat.init_drops(wl["drops"], W=10.0)
        lat.set_measure(0, wl["n_sectors"])
        info = lat.info()
        ser = lat.step(steps, measure_every=every, cap=steps // every + 1)
        a = ser[-1]
        sec = np.array([a.sector_deg[k] for k in range(a.n_sectors)], dtype=np.float64)
        sol = wl["solids"][0]
        app, D, Rd = apparent_angle(lat.rho, lat.read(G.FIELD_CLASS), info["rho_m"], sol["center"], sol["radius"])
        lat.close()
        r = dict(mu_w=m, theta=float(a.mean_deg) if a.status == 0 else math.nan, n_valid=int(a.n_valid),
                 sector_spread=float(np.nanmax(sec) - np.nanmin(sec)) if a.n_valid else math.nan,
                 drift=float(abs(ser[-1].mean_deg - ser[-2].mean_deg)) if len(ser) > 1 else math.nan,
                 apparent=float(app), drop_radius=float(Rd) if Rd is not None else math.nan)
        res.append(r)
        log(f"sessile3d {wall}: mu_w {m}: theta {r['theta']:.2f} (spread {r['sector_spread']:.2f}), "
            f"apparent {r['apparent']:.2f}, {time.perf_counter() - t0:.1f} s")
    return dict(kind="sessile3d", wall=wall, n=n, steps=steps, cases=res)


def main(argv=None):
    ap = argparse.ArgumentParser(description="wettability / drop-size / curvature sweeps on the batched solver")
    ap.add_argument("kind", choices=("wettability", "size", "curvature", "gravity", "sc-wettability", "pf-wettability",
                                     "sessile3d"))
    ap.add_argument("--Tr", type=float, default=0.6)
    ap.add_argument("--f64", action="store_true", help="FP64 storage and arithmetic (default FP32 storage)")
    ap.add_argument("--scale", type=float, default=1.0, help="every length times this (1: the 700 x 400 lattice)")
    ap.add_argument("--k", type=float, default=0.28, help="EOS scaling k (a smaller k widens the interface)")
    ap.add_argument("--kappa", type=float, default=0.01)
    ap.add_argument("--mu", type=float, nargs="*", default=None, help="wall chemical potentials (default per sweep)")
    ap.add_argument("--g", type=float, default=0.0, help="gravity toward the floor (negative: pendent drops)")
    ap.add_argument("--g-start", type=int, default=20000, help="first step with gravity")
    ap.add_argument("--wall", choices=("halfway", "interpolated"), default="halfway",
                    help="curved-wall scheme: halfway bounce-back, or the interpolated one with the mass correction")
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=0.02)
    ap.add_argument("--min-steps", type=int, default=10000)
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.kind == "sessile3d":
        rep = sessile3d(wall=a.wall, log=log, **({"steps": a.max_steps} if a.max_steps != 200000 else {}))
        print(json.dumps({k: v for k, v in rep.items() if k != "cases"}), flush=True)
        for r in rep["cases"]:
            print(json.dumps(r), flush=True)
        return 0
    if a.kind in ("sc-wettability", "pf-wettability"):
        rep = (sc_wettability if a.kind == "sc-wettability" else pf_wettability)(log=log)
        print(json.dumps({k: v for k, v in rep.items() if k != "cases"}), flush=True)
        for r in rep["cases"]:
            print(json.dumps(r), flush=True)
        return 0
    rep = run(a.kind, Tr=a.Tr, precision=G.LBM_F64 if a.f64 else G.LBM_F32, scale=a.scale, every=a.every,
              tol=a.tol, min_steps=a.min_steps, max_steps=a.max_steps, k=a.k, kappa=a.kappa, g=a.g,
              g_start=a.g_start if a.g else 0,
              mu=tuple(a.mu) if a.mu else None, log=log,
              bc_mode=G.LBM_BC_BOUZIDI_MC if a.wall == "interpolated" else G.LBM_BC_HALFWAY)
    print(json.dumps({k: v for k, v in rep.items() if k != "cases"}), flush=True)
    for r in rep["cases"]:
        print(json.dumps(r), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
