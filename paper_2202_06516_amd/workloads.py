"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds inputs only -- lattice sizes, solid and drop placements,
wettability values and seeded synthetic fields -- and none of the method's
arithmetic (no equation of state, collision, streaming or measurement).  Both
the GPU library and the CPU oracle receive what it produces.

Workloads (the paper's drops on curved solids, Sec. IV; no dataset exists):
  sessile_2d   D2Q9 FP64 128x128 periodic, cylinder r=24 at (64,40), drop r0=20
               tangent on top at (64,84), 5000 steps, angle every 100 steps
  sessile_3d   D3Q19 FP32 256^3 walled box, sphere r=60 at (128,128,92), drop
               r0=40 tangent on top at (128,128,192), 20000 steps, Tr=0.8 (the
               paper's second temperature; the three-dimensional lattice is not
               stable at Tr=0.6 with this forcing)
  striped_3d   D3Q19 FP32 512^3 walled box, sphere r=120 with latitude stripes
               (width 16) of two wettabilities, sessile or pendent drop r0=80,
               gravity 1e-6 .. 1e-5 lu
  cavity_2d    D2Q9 128x128 periodic, circular cavity r=56 at the centre, drop
               r0=20 at its lowest point (concave substrate)
  cavity_3d    D3Q19 64^3, spherical cavity r=28 at the centre, drop r0=16
  bump_case    a drop on a circular bump of radius R and height H above a
               walled floor (Fig. 2a); sweep_cases builds the wettability,
               drop-size and curvature sweeps of Sec. IV A-B from it
  sc_sessile_2d  the sessile layout for the pseudopotential model (wall density
               rho_w in place of mu_w)
  pf_sessile_2d / pf_sessile_3d  the sessile layout for the phase-field model
               (order parameter +1 liquid, -1 gas; wall order parameter phi_w
               in place of mu_w), a channel or box walled as stated
  batch_cases  many D2Q9 drops on cylinders of random sizes (batched solver)
  warmstart_cases  256^2 D2Q9 drops on cylinders, cylinder radius 16..64, drop
               radius 18..48 (smaller drops dissolve into the gas at Tr=0.8
               before they settle), mu_w -0.01..0.1 (learned warm start)
"""
from __future__ import annotations

import numpy as np

# wall chemical potentials of the paper's wettability sweep (Sec. IV C)
MU_W_SWEEP = (-0.01, 0.04, 0.1)


def sessile_2d(mu_w=0.04, n=128, scale=1.0):
    """Cylinder + tangent drop on a periodic square lattice (scaled with n/128)."""
    s = n / 128.0 * scale
    return dict(dim=2, n=(n, n), wall=(0, 0), Tr=0.6,
                solids=[dict(center=(64 * s, 40 * s), radius=24 * s, mu_w=mu_w)],
                drops=[((64 * s, 84 * s), 20 * s)], steps=5000, every=100)


def sessile_3d(mu_w=0.04, n=256):
    """Sphere + tangent drop in a walled cube (the 256^3 layout, scaled with n/256)."""
    s = n / 256.0
    cz = 92 * s
    R = 60 * s
    r0 = 40 * s
    return dict(dim=3, n=(n, n, n), wall=(1, 1, 1), Tr=0.8,
                solids=[dict(center=(128 * s, 128 * s, cz), radius=R, mu_w=mu_w)],
                drops=[((128 * s, 128 * s, cz + R + r0), r0)], steps=20000, every=500, n_sectors=32)


def striped_3d(n=512, pendent=False, g=1e-6, mu1=-0.0183, mu2=0.0700, width=16.0):
    """Sphere with latitude stripes; sessile (drop above) or pendent (drop below)."""
    s = n / 512.0
    R, r0 = 120 * s, 80 * s
    if pendent:
        cz = 336 * s
        drop = ((256 * s, 256 * s, cz - R - r0), r0)
        gv = (0.0, 0.0, -g)
    else:
        cz = 176 * s
        drop = ((256 * s, 256 * s, cz + R + r0), r0)
        gv = (0.0, 0.0, -g)
    return dict(dim=3, n=(n, n, n), wall=(1, 1, 1), Tr=0.8,
                solids=[dict(center=(256 * s, 256 * s, cz), radius=R, stripes=(mu1, mu2, width * s))],
                drops=[drop], g=gv, g_start=10000, steps=50000, every=500, n_sectors=64)


def wedge_density(shape, center, R, theta0_deg, rho_m, rho_lo, rho_hi, slope=0.05, half_chord=30.0,
                  top=40.0, side=90.0, floor=10.0):
    """Synthetic 2-D liquid region meeting a circle at a prescribed angle.

    The liquid is bounded by two straight lines through the points of the
    circle (center, R) at +-half_chord from the vertical axis, each at angle
    theta0 to the circle's tangent measured through the liquid, plus a flat top,
    a floor floor lu above the centre (so the lines' second crossings of the
    circle stay dry) and two far side walls.  The density is rho_m + slope * s, with s the
    minimum of the signed distances to these lines (positive inside), clipped
    to [rho_lo, rho_hi].  Along any lattice link near a contact point the
    density is affine, so isodensity crossings lie exactly on the line.
    Returns an array of shape (1, ny, nx).
    """
    _, ny, nx = shape
    cx, cy = center
    phi = np.arcsin(half_chord / R)
    th = np.deg2rad(theta0_deg)
    lines = []  # (point, inward unit normal)
    for side_sign in (1.0, -1.0):
        px, py = cx + side_sign * R * np.sin(phi), cy + R * np.cos(phi)
        # tangent toward the axis and outward normal at the contact point
        tx, ty = -side_sign * np.cos(phi), np.sin(phi)
        nx_, ny_ = side_sign * np.sin(phi), np.cos(phi)
        # interface direction: rotate t toward n by theta0
        vx, vy = np.cos(th) * tx + np.sin(th) * nx_, np.cos(th) * ty + np.sin(th) * ny_
        # inward normal of the line: the side containing the tangent direction t
        mx, my = -vy, vx
        if mx * tx + my * ty < 0:
            mx, my = -mx, -my
        lines.append((px, py, mx, my))
    ytop = cy + R + top
    lines.append((cx, ytop, 0.0, -1.0))
    lines.append((cx, cy + floor, 0.0, 1.0))
    lines.append((cx - side, cy, 1.0, 0.0))
    lines.append((cx + side, cy, -1.0, 0.0))
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    s = np.full((ny, nx), np.inf)
    for px, py, mx, my in lines:
        s = np.minimum(s, (xx - px) * mx + (yy - py) * my)
    rho = np.clip(rho_m + slope * s, rho_lo, rho_hi)
    return rho[None, :, :]


def cavity_wedge_density(shape, center, R, theta0_deg, rho_m, rho_lo, rho_hi, slope=0.05, half_chord=30.0,
                         top=40.0):
    """Synthetic 2-D liquid pool at the bottom of a circular cavity, meeting the
    cavity wall at a prescribed angle (the concave case of Fig. 2b).

    The liquid is bounded by two straight lines through the wall points at
    +-half_chord from the vertical axis, below the centre, each at angle theta0
    to the wall's tangent measured through the liquid, and by a flat top top lu
    above the cavity's lowest point.  The lines rise toward the axis only if
    theta0 exceeds the half-angle of the chord, asin(half_chord / R).  The
    density is rho_m + slope * s, s the minimum of the signed distances to
    these lines (positive inside), clipped to [rho_lo, rho_hi].
    Returns an array of shape (1, ny, nx).
    """
    _, ny, nx = shape
    cx, cy = center
    phi = np.arcsin(half_chord / R)
    th = np.deg2rad(theta0_deg)
    lines = []  # (point, inward unit normal)
    for side_sign in (1.0, -1.0):
        px, py = cx + side_sign * R * np.sin(phi), cy - R * np.cos(phi)
        # tangent toward the axis (down the wall) and wall normal into the fluid
        tx, ty = -side_sign * np.cos(phi), -np.sin(phi)
        nx_, ny_ = -side_sign * np.sin(phi), np.cos(phi)
        vx, vy = np.cos(th) * tx + np.sin(th) * nx_, np.cos(th) * ty + np.sin(th) * ny_
        mx, my = -vy, vx
        if mx * tx + my * ty < 0:
            mx, my = -mx, -my
        lines.append((px, py, mx, my))
    lines.append((cx, cy - R + top, 0.0, -1.0))
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    s = np.full((ny, nx), np.inf)
    for px, py, mx, my in lines:
        s = np.minimum(s, (xx - px) * mx + (yy - py) * my)
    rho = np.clip(rho_m + slope * s, rho_lo, rho_hi)
    return rho[None, :, :]


def plane_film_density(shape, rho_m, rho_lo, rho_hi, heights, x_split, liquid_above=True, slope=0.5, far=14.0):
    """Synthetic 3-D liquid bounded by a horizontal plane, for measurements on a
    sphere: liquid above z = h (liquid_above) or below it, up to a far plane
    far lu beyond.  heights = (h_left, h_right): the plane is at h_left for
    x < x_split - 3, at h_right for x > x_split + 3, and between them linear in
    x.  The density is rho_m + slope * s, s the signed distance-like quantity
    min(+-(z - h(x)), far - +-(z - h(x))) (positive in the liquid), clipped to
    [rho_lo, rho_hi]; away from the x band it is affine in z, so along every
    lattice link isodensity crossings lie on the plane.  Returns an array of
    shape (nz, ny, nx)."""
    nz, ny, nx = shape
    zz, _, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                            np.arange(nx, dtype=np.float64), indexing="ij")
    hl, hr = heights
    t = np.clip((xx - (x_split - 3.0)) / 6.0, 0.0, 1.0)
    h = hl + (hr - hl) * t
    sgn = 1.0 if liquid_above else -1.0
    s = sgn * (zz - h)
    s = np.minimum(s, far - s)
    return np.clip(rho_m + slope * s, rho_lo, rho_hi)


def cavity_2d(mu_w=0.04, n=128):
    """Drop resting at the bottom of a circular cavity (concave substrate,
    Fig. 2b) on a square lattice: cavity radius 7n/16 at the centre, drop
    radius 5n/32 touching the wall from inside at the lowest point."""
    s = n / 128.0
    R, r0 = 56 * s, 20 * s
    c = (64 * s, 64 * s)
    return dict(dim=2, n=(n, n), wall=(0, 0), Tr=0.6,
                solids=[dict(center=c, radius=R, mu_w=mu_w, cavity=True)],
                drops=[((c[0], c[1] - R + r0), r0)], steps=5000, every=100)


def cavity_3d(mu_w=0.04, n=64):
    """Drop at the bottom of a spherical cavity in a cube (D3Q19, Tr = 0.8):
    cavity radius 7n/16 at the centre, drop radius n/4 touching it from inside."""
    s = n / 64.0
    R, r0 = 28 * s, 16 * s
    c = (32 * s, 32 * s, 32 * s)
    return dict(dim=3, n=(n, n, n), wall=(0, 0, 0), Tr=0.8,
                solids=[dict(center=c, radius=R, mu_w=mu_w, cavity=True)],
                drops=[((c[0], c[1], c[2] - R + r0), r0)], steps=5000, every=100, n_sectors=16)


def bump_case(nx, ny, R, H, r0, mu_w):
    """A drop on a circular bump (Fig. 2a): the arc of a circle of radius R rising
    H above a flat floor, centred horizontally, with the drop of radius r0
    tangent on its top.  For a lattice walled along y (two solid layers at each
    end, the floor surface at y = 1.5 lu); the bump's width is
    L = 2 sqrt(2 R H - H^2)."""
    floor = 1.5
    cy = floor + H - R
    return dict(n=(int(nx), int(ny)), solid=dict(center=(nx / 2.0, cy), radius=float(R), mu_w=float(mu_w)),
                drop=((nx / 2.0, floor + H + r0), float(r0)))


# the sweeps of Sec. IV A-B on bumps (lattice 700 x 400 walled along y, as the
# paper's gravity-free domain): wettability at r0 = 40 on R = 150, drop size
# r0 = 30..100 on R = 400, curvature R = 150..400 at r0 = 40; all with H = 100.
# Below mu_w = -0.02 a drop of r0 = 40 spreads to the foot of the bump at Tr = 0.6.
SWEEP_MU = tuple(float(m) for m in np.round(np.linspace(-0.02, 0.16, 10), 4))
SWEEP_MU5 = (-0.01, 0.02, 0.04, 0.07, 0.1)
SWEEP_R0 = (30, 40, 50, 60, 70, 80, 90, 100)
SWEEP_RS = (150, 200, 250, 300, 350, 400)
SWEEP_MU3 = (-0.01, 0.04, 0.1)            # the paper's 70 / 100 / 140 degree surfaces (Sec. IV C)
SWEEP_R0_GRAVITY = (20, 35, 50, 65, 80, 95)


def sweep_cases(kind, scale=1.0, mu=None, values=None):
    """Case table of one sweep ("wettability", "size", "curvature" or "gravity") with a
    (value, mu_w) label per case; every length (lattice, H, R, r0) times scale."""
    s = float(scale)
    nx, ny, H = int(round(700 * s)), int(round(400 * s)), 100.0 * s
    if kind == "wettability":
        mu = SWEEP_MU if mu is None else mu
        pairs = [(m, m) for m in mu]
        cases = [bump_case(nx, ny, 150.0 * s, H, 40.0 * s, m) for m in mu]
    elif kind == "size":
        mu = SWEEP_MU5 if mu is None else mu
        values = SWEEP_R0 if values is None else values
        pairs = [(r, m) for m in mu for r in values]
        cases = [bump_case(nx, ny, 400.0 * s, H, r * s, m) for r, m in pairs]
    elif kind == "gravity":
        # sessile (or, with gravity reversed, pendent) drops of growing size on
        # the wide bump: the Bond number grows as r0^2 (Sec. IV C)
        mu = SWEEP_MU3 if mu is None else mu
        values = SWEEP_R0_GRAVITY if values is None else values
        pairs = [(r, m) for m in mu for r in values]
        cases = [bump_case(nx, ny, 400.0 * s, H, r * s, m) for r, m in pairs]
    elif kind == "curvature":
        mu = SWEEP_MU5 if mu is None else mu
        values = SWEEP_RS if values is None else values
        pairs = [(R, m) for m in mu for R in values]
        cases = [bump_case(nx, ny, R * s, H, 40.0 * s, m) for R, m in pairs]
    else:
        raise ValueError(kind)
    return cases, pairs


# the pseudopotential (Shan-Chen) model: psi = 1 - exp(-rho), interaction
# strength G, and the bulk densities of a flat interface it relaxes to (a
# converged 128 x 4 slab of the oracle, MRT and BGK alike to 4e-5)
SC_G = -6.0
SC_RHO_L = 2.649
SC_RHO_G = 0.0735


def sc_sessile_2d(rho_w=0.8, n=128):
    """The sessile layout of sessile_2d for the pseudopotential model: cylinder
    r = 24 at (64, 40), drop r0 = 20 on top, interface width W = 5, wall
    density rho_w on the cylinder (scaled with n/128)."""
    s = n / 128.0
    return dict(dim=2, n=(n, n), wall=(0, 0), model=1,
                solids=[dict(center=(64 * s, 40 * s), radius=24 * s, mu_w=rho_w)],
                drops=[((64 * s, 84 * s), 20 * s)], W=5.0, steps=5000, every=100)


# the phase-field model's parameters (both sides receive exactly these): interface
# width xi = sqrt(2 kappa / A) = 2, so that the Eq. 16 profile of width W = 2 xi
# is the flat-interface profile tanh(r / xi)
PF_PARAMS = dict(pf_A=0.01, pf_kappa=0.02, pf_gamma=1.0, pf_tau=1.0, pf_rho0=1.0)
PF_W = 4.0


def pf_sessile_2d(phi_w=0.3, n=(96, 64)):
    """Phase-field model: a disc in a channel walled along y, drop tangent on top."""
    c, R, r0 = (47.7, 22.3), 12.4, 9.0
    return dict(dim=2, n=n, wall=(0, 1), model=2, W=PF_W,
                solids=[dict(center=c, radius=R, mu_w=phi_w)],
                drops=[((47.5, c[1] + R + r0), r0)], every=100)


def pf_sessile_3d(phi_w=0.3, n=(64, 48, 48)):
    """Phase-field model: a sphere in a walled box, drop tangent on top."""
    c, R, r0 = (31.6, 24.2, 16.3), 9.4, 8.0
    return dict(dim=3, n=n, wall=(1, 1, 1), model=2, W=PF_W,
                solids=[dict(center=c, radius=R, mu_w=phi_w)],
                drops=[((31.6, 24.2, c[2] + R + r0), r0)], every=100, n_sectors=16)


def random_state_perturbation(shape, q, seed, amplitude=1e-3):
    """Seeded multiplicative noise factors (1 + a*U(-1,1)) for populations [q, *shape]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(q,) + tuple(shape))


def batch_cases(n_cases=512, seed=0, nmin=64, nmax=512, rs=(16.0, 128.0), r0=(12.0, 96.0),
                mu=(-0.01, 0.1), W=10.0, max_tries=100):
    """Case table of independent 2-D drops on cylinders (seeded PCG64).

    Sides uniform in [nmin, nmax]; cylinder radius, drop radius and wall
    chemical potential uniform in the given ranges.  A draw is feasible if
    2 R_s + 2 r0 + 2 W + 8 <= ny and 2 max(R_s, r0) + 8 <= nx; infeasible
    draws are redrawn up to max_tries times, then both radii are scaled down.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = []
    accepted = 0
    for _ in range(n_cases):
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        ok = False
        for _t in range(max_tries):
            Rs = float(rng.uniform(*rs))
            rd = float(rng.uniform(*r0))
            muw = float(rng.uniform(*mu))
            if 2 * Rs + 2 * rd + 2 * W + 8 <= ny and 2 * max(Rs, rd) + 8 <= nx:
                ok = True
                break
        if ok:
            accepted += 1
        else:
            f = min((ny - 2 * W - 8) / (2 * Rs + 2 * rd), (nx - 8) / (2 * max(Rs, rd)))
            Rs, rd = Rs * f, rd * f
        cy = W + 4 + Rs
        cases.append(dict(n=(nx, ny), solid=dict(center=(nx / 2.0, cy), radius=Rs, mu_w=muw),
                          drop=((nx / 2.0, cy + Rs + rd), rd)))
    return cases, accepted / n_cases


# seed offsets of the disjoint warm-start sets (training, validation, test)
WARM_SEEDS = dict(train=1000, val=2000, test=3000)


def pf_batch_cases(cases, seed, phi_w=(-0.4, 0.4)):
    """The case table for the phase-field model: the same layouts, the wall value
    of each solid a wall order parameter uniform in phi_w (seeded PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [dict(c, solid=dict(c["solid"], mu_w=float(rng.uniform(*phi_w)))) for c in cases]


def warmstart_cases(n_cases, seed, side=256, rs=(16.0, 64.0), r0=(18.0, 48.0), mu=(-0.01, 0.1), W=10.0):
    """Drops on cylinders for the learned warm start (seeded PCG64).

    A side x side periodic D2Q9 lattice; cylinder radius, drop radius and
    wall chemical potential uniform in the given ranges; the cylinder is
    centred horizontally with its lowest point W + 4 above the bottom row and
    the drop (Eq. 16 profile) tangent on top.  Returns the case table.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    cases = []
    for _ in range(n_cases):
        Rs = float(rng.uniform(*rs))
        rd = float(rng.uniform(*r0))
        muw = float(rng.uniform(*mu))
        cy = W + 4 + Rs
        cases.append(dict(n=(side, side), solid=dict(center=(side / 2.0, cy), radius=Rs, mu_w=muw),
                          drop=((side / 2.0, cy + Rs + rd), rd)))
    return cases
