"""A drop sliding on a tilted curved plate: dynamic contact angle hysteresis (Sec. IV D, Fig. 9-11).

Reading of the set-up (the paper gives the drop, r0 = 100, the slope, 20
degrees, the intrinsic angle, 120 degrees, and a 3000 lu long domain, not the
plate's shape): the plate is the arc of a circle of radius R rising H above a
walled floor (the bump of Fig. 2a) with R much larger than the drop, and the
slope is applied by tilting gravity by phi, g = |g| (sin phi, -cos phi), the
lattice staying axis-aligned; the box is walled on all sides.  The drop first relaxes without gravity
(g_start_step), then slides along the arc.  With ``stripes`` the plate is
chemically patterned: bands of arc length ``width`` alternating mu_w1 / mu_w2
from the top of the arc (Fig. 9).

Every ``every`` steps the in-step measurement gives the advancing angle (on
the side the tangential part of g points to), the receding angle and both
contact points.  The summary over the sliding phase: range (max - min) and
standard deviation of theta_A and theta_R, and the hysteresis theta_A -
theta_R (mean, max, share of samples within 5 degrees).  With ``young`` the
unbalanced Young force (Sec. IV E, Eq. 17-18) of both contact lines is taken
after every chunk of steps as well (Fig. 13-14).

Command line: ``python -m paper_2202_06516_amd.rolling --help``.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbm as G


def start_drop(cx, cy, R, x0, r0):
    """Centre of a drop of radius r0 touching the arc at abscissa x0 from above."""
    ys = cy + math.sqrt(R * R - (x0 - cx) ** 2)
    nx_, ny_ = (x0 - cx) / R, (ys - cy) / R
    return (x0 + r0 * nx_, ys + r0 * ny_)


def run(nx=3000, ny=400, R=6000.0, H=100.0, r0=100.0, x0=900.0, mu_w=0.1, stripes=None, g=5e-7, phi_deg=20.0,
        Tr=0.6, relax=20000, steps=600000, every=500, chunk=10000, stop_frac=0.6, precision=G.LBM_F32,
        young=None, log=print):
    """young = (gamma, theta_1, theta_2): also the unbalanced Young force of
    Eq. 17 on both contact lines at every measurement, taken inside the step
    loop (lbm_set_young: theta_eq of Eq. 18 from the footprint on the two kinds
    of band)."""
    phi = math.radians(phi_deg)
    # a closed box: with the tilted gravity an open (periodic) x axis would let
    # the whole gas column accelerate along x without bound
    lat = G.Lattice(G.LBM_D2Q9, n=(nx, ny, 1), precision=precision, axis_bc=(1, 1, 0), tau=1.0, Tr=Tr, k=0.28,
                    kappa=0.01, g=(g * math.sin(phi), -g * math.cos(phi), 0.0), g_start_step=relax)
    cx, cy = nx / 2.0, 1.5 + H - R
    sol = dict(center=(cx, cy), radius=R, pole=(0.0, 1.0))
    if stripes is None:
        sol["mu_w"] = mu_w
    else:
        sol["stripes"] = tuple(stripes)
    lat.set_solids([sol])
    lat.init_drops([(start_drop(cx, cy, R, x0, r0), r0)], W=10.0)
    lat.set_measure(0, 2)
    if young is not None:
        lat.set_young(*young)
    half = math.sqrt(2 * R * H - H * H)       # half-width of the arc above the floor
    x_stop = cx + stop_frac * half
    recs, forces = [], []
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        series = lat.step(n, measure_every=every, cap=n // every + 1)
        if young is not None:
            for a, y in zip(series, lat.young_series(cap=max(1, len(series)))):
                if a.status == 0 and y.status == 0 and math.isfinite(y.force[0]) and math.isfinite(y.force[1]):
                    k = 0 if a.contact[0][0] > a.contact[1][0] else 1
                    # Eq. 17 per line is gamma (cos theta - cos theta_eq); the force on a line points out of the
                    # drop, so projected on +x (right positive, Sec. IV E) the right (advancing) line takes
                    # -gamma (cos theta_A - cos theta_eq) and the left (receding) line +gamma (cos theta_R - ...)
                    forces.append(dict(step=int(a.step), force_a=-float(y.force[k]), force_r=float(y.force[1 - k]),
                                       theta_eq_a=float(y.theta_eq_deg[k]), theta_eq_r=float(y.theta_eq_deg[1 - k]),
                                       phi_a=float(y.phi_d[k]), phi_r=float(y.phi_d[1 - k])))
        for a in series:
            if a.status != 0:
                recs.append(dict(step=int(a.step), status=int(a.status)))
                continue
            # the advancing side is downhill: the contact point further along +x
            k = 0 if a.contact[0][0] > a.contact[1][0] else 1
            recs.append(dict(step=int(a.step), status=0, theta_a=float(a.sector_deg[k]),
                             theta_r=float(a.sector_deg[1 - k]), x_a=float(a.contact[k][0]),
                             x_r=float(a.contact[1 - k][0]),
                             library_sides=bool(a.adv_deg == a.sector_deg[k] and a.rec_deg == a.sector_deg[1 - k])))
        done += n
        last = next((r for r in reversed(recs) if r["status"] == 0), None)
        if (done // chunk) % max(1, 50000 // chunk) == 0:
            log(f"rolling: step {done}, {time.perf_counter() - t0:.1f} s, "
                f"advancing contact x = {last['x_a'] if last else float('nan'):.1f}")
        if last and done > relax and max(last["x_a"], last["x_r"]) > x_stop:
            break
    seconds = time.perf_counter() - t0
    inf = lat.info()
    lat.close()
    slide = [r for r in recs if r["status"] == 0 and r["step"] > relax]
    out = dict(nx=nx, ny=ny, R=R, H=H, r0=r0, mu_w=mu_w if stripes is None else None, stripes=stripes, g=g, phi_deg=phi_deg, Tr=Tr,
               steps=done, seconds=round(seconds, 2),
               mlups=round(float(inf["n_fluid"]) * done / seconds / 1e6, 1), records=recs)
    fs = [f for f in forces if f["step"] > relax]
    if young is not None and len(fs) >= 2:
        fa = np.array([f["force_a"] for f in fs])
        fr = np.array([f["force_r"] for f in fs])
        out.update(young=list(young), forces=forces, force_a_mean=round(float(fa.mean()), 5),
                   force_r_mean=round(float(fr.mean()), 5), force_a_range=[round(float(fa.min()), 5), round(float(fa.max()), 5)],
                   force_r_range=[round(float(fr.min()), 5), round(float(fr.max()), 5)],
                   force_r_largest_jump=round(float(np.max(np.abs(np.diff(fr)))), 5))
    if len(slide) >= 2:
        ta = np.array([r["theta_a"] for r in slide])
        tr = np.array([r["theta_r"] for r in slide])
        xa = np.array([r["x_a"] for r in slide])
        out.update(library_sides=all(r["library_sides"] for r in slide), travel=round(float(xa[-1] - xa[0]), 1),
                   theta_a_range=round(float(ta.max() - ta.min()), 2),
                   theta_r_range=round(float(tr.max() - tr.min()), 2),
                   hysteresis_mean=round(float(np.mean(ta - tr)), 2), hysteresis_max=round(float(np.max(ta - tr)), 2),
                   hysteresis_within_5deg=round(float(np.mean(np.abs(ta - tr) <= 5.0)), 3),
                   theta_a_std=round(float(ta.std()), 2), theta_r_std=round(float(tr.std()), 2),
                   theta_a_mean=round(float(ta.mean()), 2), theta_r_mean=round(float(tr.mean()), 2))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="drop sliding on a tilted curved plate (dynamic hysteresis)")
    ap.add_argument("--nx", type=int, default=3000)
    ap.add_argument("--ny", type=int, default=400)
    ap.add_argument("--R", type=float, default=6000.0)
    ap.add_argument("--H", type=float, default=100.0)
    ap.add_argument("--r0", type=float, default=100.0)
    ap.add_argument("--x0", type=float, default=900.0)
    ap.add_argument("--mu", type=float, default=0.1, help="wall chemical potential (homogeneous plate)")
    ap.add_argument("--stripes", type=float, nargs=3, default=None, metavar=("MU1", "MU2", "WIDTH"))
    ap.add_argument("--g", type=float, default=5e-7)
    ap.add_argument("--phi", type=float, default=20.0)
    ap.add_argument("--Tr", type=float, default=0.6)
    ap.add_argument("--relax", type=int, default=20000)
    ap.add_argument("--steps", type=int, default=600000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--chunk", type=int, default=10000, help="steps between host checks (and Young-force samples)")
    ap.add_argument("--young", type=float, nargs=3, default=None, metavar=("GAMMA", "THETA1", "THETA2"),
                    help="also the unbalanced Young force (Eq. 17-18) at every measurement")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    rep = run(nx=a.nx, ny=a.ny, R=a.R, H=a.H, r0=a.r0, x0=a.x0, mu_w=a.mu, stripes=a.stripes, g=a.g,
              phi_deg=a.phi, Tr=a.Tr, relax=a.relax, steps=a.steps, every=a.every, chunk=a.chunk,
              young=tuple(a.young) if a.young else None, log=log)
    print(json.dumps({k: v for k, v in rep.items() if k not in ("records", "forces")}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
