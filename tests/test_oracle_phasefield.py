"""Pins of the oracle's phase-field model (Sec. V names phase-field models as
a third family the measurement applies to).

The model: an order parameter phi (liquid +1, gas -1) with the free energy
A/4 (phi^2 - 1)^2 + kappa/2 |grad phi|^2, carried by a second population set
whose equilibrium gives the Cahn-Hilliard equation; the capillary force
mu grad(phi) on the fluid populations; wetting by a wall order parameter on
the two solid layers.  What the mathematics fixes:

- a flat interface at rest is phi = tanh(x / xi), xi = sqrt(2 kappa / A),
  between bulk phases at exactly +-1 with mu = 0;
- Laplace's law with the surface tension of that profile,
  sigma = (2 sqrt 2 / 3) sqrt(kappa A);
- the order parameter and the mass are conserved to round-off, walls and a
  curved solid included;
- the model is odd in phi: negating phi and the wall value negates phi, mu
  and the order-parameter populations bit for bit and leaves the fluid
  populations unchanged;
- one step equals the step written out by its definitions on a small
  lattice with walls and a disc.
"""
import math

import numpy as np
import pytest

import oracle as O

from .test_oracle_pins import _brute_lattice

PF = dict(model=2, bgk=1, tau=1.0, pf_A=0.01, pf_kappa=0.02, pf_gamma=1.0, pf_tau=1.0, pf_rho0=1.0)
XI = math.sqrt(2 * PF["pf_kappa"] / PF["pf_A"])
SIGMA = 2.0 * math.sqrt(2.0) / 3.0 * math.sqrt(PF["pf_kappa"] * PF["pf_A"])


def test_flat_interface_is_the_tanh_profile():
    o = O.Oracle(2, (128, 4), (0, 0), **PF)
    x = np.arange(128.0)
    o.set_rho(np.broadcast_to(np.tanh((x - 43.5) / XI) * np.tanh((83.5 - x) / XI), (1, 4, 128)))
    o.step(2000)
    o.update_derived()
    phi = o.phi[0, 0]
    assert abs(phi[63] - 1.0) < 1e-4 and abs(phi[0] + 1.0) < 1e-4
    assert np.abs(o.mu).max() < 1e-5
    # the fourth-order stencils resolve an interface of xi = 2 lattice units to a few 1e-3
    assert np.max(np.abs(phi[30:58] - np.tanh((x[30:58] - 43.5) / XI))) < 5e-3


@pytest.mark.parametrize("R,tol", [(16.0, 0.03), (22.0, 0.02)])
def test_laplace_law(R, tol):
    # mechanical balance grad(rho cs^2) = mu grad(phi): the pressure jump of a
    # free drop times its radius is the surface tension of the flat profile
    n = 96
    yy, xx = np.mgrid[0:n, 0:n].astype(float)
    o = O.Oracle(2, (n, n), (0, 0), **PF)
    o.set_rho((-np.tanh((np.hypot(xx - 47.5, yy - 47.5) - R) / XI))[None])
    o.step(6000)
    o.update_derived()
    dp = (o.rho[0, 48, 48] - o.rho[0, 0, 0]) / 3.0
    assert abs(dp * R / SIGMA - 1.0) < tol, (R, dp * R, SIGMA)


def _drop_on_disc(phi_w, negate=False, n=(64, 48)):
    # a drop (Eq. 16 profile with the width of the flat interface) resting on a
    # disc in a channel walled along y; negate: the order parameter and the wall
    # value of the same state negated
    o = O.Oracle(2, n, (0, 1), **PF)
    o.add_sphere((31.7, 14.3), 9.4, mu_w=-phi_w if negate else phi_w)
    o.init_drops([(31.5, 30.0)], [8.0], W=2 * XI)
    if negate:
        o.set_rho(-o.phi)
    return o


def test_phi_and_mass_conserved():
    o = _drop_on_disc(0.3)
    o.update_derived()
    fl = o.cls == 0
    p0, m0 = o.phi[fl].sum(), o.mass()
    o.step(400)
    o.update_derived()
    assert abs(o.phi[fl].sum() - p0) < 1e-12 * np.abs(o.phi[fl]).sum()
    assert abs(o.mass() / m0 - 1.0) < 1e-12


def test_model_is_odd_in_phi():
    a = _drop_on_disc(0.3)
    b = _drop_on_disc(0.3, negate=True)
    assert np.array_equal(a.phi, -b.phi)
    a.step(300)
    b.step(300)
    a.update_derived()
    b.update_derived()
    assert np.array_equal(a.phi, -b.phi) and np.array_equal(a.f, b.f)
    assert np.array_equal(a.mu, -b.mu) and np.array_equal(a.g, -b.g)


def test_wall_order_parameter_sets_the_wetting():
    # a wall preferring the liquid (phi_w > 0) wets more: the angle falls as phi_w rises
    th = []
    for pw in (-0.4, 0.0, 0.4):
        o = _drop_on_disc(pw)
        o.step(3000)
        th.append(o.measure(0, 2).mean_deg)
    assert th[0] > th[1] > th[2], th
    assert 70.0 < th[1] < 110.0, th


def _brute_pf_step(f, g, prm, disc, phi_w, wall_phi, size, wall):
    """One phase-field step by its definitions, node by node (D2Q9): classes
    (disc or the two outer layers of a wall axis; first layer = solid with a
    fluid neighbour, second = solid with a first-layer one), phi = sum g on
    fluid, on both layers phi_w (the disc's) or wall_phi (the walls'),
    mu = A (phi^3 - phi) - kappa lap4(phi),
    F = mu grad4(phi), BGK with exact-difference forcing for f, BGK toward the
    Cahn-Hilliard equilibrium for g, pull streaming with halfway bounce-back."""
    e, w = _brute_lattice(2)
    Q = 9
    opp = [int(np.nonzero((e == -e[i]).all(1))[0][0]) for i in range(Q)]
    nx, ny = size

    def wrap(p):
        q = list(p)
        for d, nd in enumerate((nx, ny)):
            if q[d] < 0 or q[d] >= nd:
                if wall[d]:
                    return None
                q[d] %= nd
        return tuple(q)

    def in_disc(p):
        c, r = disc
        return (p[0] - c[0]) ** 2 + (p[1] - c[1]) ** 2 <= r * r

    def solid(p):
        return in_disc(p) or any(wall[d] and (p[d] < 2 or p[d] >= nd - 2) for d, nd in enumerate((nx, ny)))

    nodes = [(x, y) for y in range(ny) for x in range(nx)]
    nb = {p: [wrap((p[0] + e[i][0], p[1] + e[i][1])) for i in range(Q)] for p in nodes}
    cls = {p: 0 if not solid(p) else (1 if any(m and not solid(m) for m in nb[p][1:]) else 3) for p in nodes}
    for p in nodes:
        if cls[p] == 3 and any(m and cls[m] == 1 for m in nb[p][1:]):
            cls[p] = 2
    fx = {p: f[:, 0, p[1], p[0]] for p in nodes}
    gx = {p: g[:, 0, p[1], p[0]] for p in nodes}
    phi = {p: gx[p].sum() if cls[p] == 0 else ((phi_w if in_disc(p) else wall_phi) if cls[p] in (1, 2) else 0.0)
           for p in nodes}

    def at(p, ax, k):
        q = [p[0], p[1]]
        q[ax] += k
        return wrap(tuple(q))

    def d1(p, ax):
        v = [phi[at(p, ax, k)] for k in (-2, -1, 1, 2)]
        return (v[0] - 8 * v[1] + 8 * v[2] - v[3]) / 12.0

    def d2(p, ax):
        v = [phi[at(p, ax, k)] for k in (-2, -1, 0, 1, 2)]
        return (-v[0] + 16 * v[1] - 30 * v[2] + 16 * v[3] - v[4]) / 12.0

    A, kap, gam, taug, tau = prm["pf_A"], prm["pf_kappa"], prm["pf_gamma"], prm["pf_tau"], prm["tau"]
    fpost, gpost = {}, {}
    for p in nodes:
        if cls[p] != 0:
            fpost[p], gpost[p] = np.zeros(Q), np.zeros(Q)
            continue
        ph = phi[p]
        mu = A * (ph ** 3 - ph) - kap * (d2(p, 0) + d2(p, 1))
        F = np.array([mu * d1(p, 0), mu * d1(p, 1), 0.0])
        r = fx[p].sum()
        j = e.T @ fx[p]
        u = j / r

        def feq(rr, uu):
            eu = e @ uu
            return w * rr * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (uu @ uu))

        fpost[p] = fx[p] - (fx[p] - feq(r, u)) / tau + feq(r, u + F / r) - feq(r, u)
        v = (j + 0.5 * F) / r
        ev = e @ v
        geq = w * (3 * gam * mu + 3 * ph * ev + ph * (4.5 * ev * ev - 1.5 * (v @ v)))
        geq[0] = ph - geq[1:].sum()
        gpost[p] = gx[p] - (gx[p] - geq) / taug
    fo, go = np.zeros_like(f), np.zeros_like(g)
    for p in nodes:
        if cls[p] != 0:
            continue
        for i in range(Q):
            src = wrap((p[0] - e[i][0], p[1] - e[i][1]))
            if src is not None and cls[src] == 0:
                fo[i, 0, p[1], p[0]] = fpost[src][i]
                go[i, 0, p[1], p[0]] = gpost[src][i]
            else:
                fo[i, 0, p[1], p[0]] = fpost[p][opp[i]]
                go[i, 0, p[1], p[0]] = gpost[p][opp[i]]
    return fo, go


def test_one_step_matches_brute_force():
    size, wall = (14, 12), (0, 1)
    disc = ((6.3, 5.6), 2.4)
    o = O.Oracle(2, size, wall, wall_mu=-0.13, **PF)
    o.add_sphere(disc[0], disc[1], mu_w=0.27)
    rng = np.random.Generator(np.random.PCG64(5))
    o.set_rho(rng.uniform(-1.0, 1.0, o.shape))
    o.step(3)                                   # non-equilibrium populations in both sets
    f, g = o.f.copy(), o.g.copy()
    fo, go = _brute_pf_step(f, g, PF, disc, 0.27, -0.13, size, wall)
    o.step(1)
    assert np.max(np.abs(o.f - fo)) < 1e-12 * np.max(np.abs(fo))
    assert np.max(np.abs(o.g - go)) < 1e-12 * np.max(np.abs(go))
