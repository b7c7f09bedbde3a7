"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: textbook
closed forms, thermodynamic identities, exact invariants of the lattice
Boltzmann step, calculus on polynomials, and geometric constructions whose
answer is known exactly.  A plausible slip in the oracle (a dropped term, a
sign, an index, a transposed operand) breaks at least one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2202_06516_amd import workloads as W

# ---------------------------------------------------------------- thermodynamics


def test_pr_critical_point_textbook():
    # Peng-Robinson textbook constants: T_c = 0.07780/0.45724 * a/(bR) to the
    # rounding of those constants, critical compressibility Z_c = 0.3074
    Tc, rc, pc = O.pr_critical()
    approx = 0.07780 / 0.45724 * O.PR_A / (O.PR_B * O.PR_R)
    assert abs(Tc / approx - 1) < 2e-4
    assert abs(pc / (rc * O.PR_R * Tc) - 0.3074) < 1e-4
    # triple root: B_c = b p_c/(R T_c) solves 64 B^3 + 6 B^2 + 12 B - 1 = 0
    B = O.PR_B * pc / (O.PR_R * Tc)
    assert abs(64 * B**3 + 6 * B**2 + 12 * B - 1) < 1e-9


def test_pr_alpha_is_one_at_tc():
    assert O.pr_alpha(1.0) == 1.0
    # omega = 0.344 (water): m = 0.37464 + 1.54226 w - 0.26992 w^2
    m = 0.37464 + 1.54226 * 0.344 - 0.26992 * 0.344**2
    assert abs(O.pr_alpha(0.6) - (1 + m * (1 - math.sqrt(0.6))) ** 2) < 1e-15


@pytest.mark.parametrize("rho", [0.01, 0.3, 2.0, 5.0, 8.5])
def test_gibbs_duhem(rho):
    # Eq. 8 differentiated: d mu / d rho = (d p0 / d rho) / rho  (Eq. 11 vs Eq. 10)
    Tc = O.pr_critical()[0]
    T, al = 0.6 * Tc, O.pr_alpha(0.6)
    h = 1e-5 * rho
    dmu = (O.pr_mu(rho + h, T, al) - O.pr_mu(rho - h, T, al)) / (2 * h)
    dp = (O.pr_p0(rho + h, T, al) - O.pr_p0(rho - h, T, al)) / (2 * h)
    assert abs(dmu - dp / rho) <= 1e-7 * abs(dp / rho) + 1e-12


@pytest.mark.parametrize("Tr", [0.6, 0.7, 0.8, 0.9])
def test_maxwell_coexistence(Tr):
    m = O.maxwell(Tr)
    Tc = O.pr_critical()[0]
    T, al = Tr * Tc, O.pr_alpha(Tr)
    pg, pl = O.pr_p0(m["rho_g"], T, al), O.pr_p0(m["rho_l"], T, al)
    ug, ul = O.pr_mu(m["rho_g"], T, al), O.pr_mu(m["rho_l"], T, al)
    assert abs(pg - pl) <= 1e-12 * max(abs(pg), 1e-12) + 1e-15
    assert abs(ug - ul) <= 1e-12
    # equal areas: the integral of (p0 - p_sat) dV vanishes, V = 1/rho
    from scipy.integrate import quad
    area, _ = quad(lambda r: (O.pr_p0(r, T, al) - m["p_sat"]) / r**2, m["rho_g"], m["rho_l"],
                   limit=400, epsabs=1e-14, epsrel=1e-12)
    assert abs(area) < 1e-8 * m["p_sat"] * (1 / m["rho_g"] - 1 / m["rho_l"])
    assert m["rho_g"] < m["rho_l"]


def _relaxed_slab(Tr, steps):
    # a flat liquid slab (y in 50..150) in gas on a periodic 6 x 200 lattice,
    # relaxed until the velocity has died out; returns the bulk liquid and gas
    # densities (slab middle, far gas) and the largest remaining speed
    ny = 200
    o = O.Oracle(2, (6, ny), Tr=Tr, k=0.28, kappa=0.01)
    inf = o.info()
    y = np.arange(ny)
    prof = inf["rho_g"] + 0.5 * (inf["rho_l"] - inf["rho_g"]) * (np.tanh((y - 50) / 3.0) - np.tanh((y - 150) / 3.0))
    o.set_rho(np.broadcast_to(prof[:, None], (ny, 6))[None].copy())
    o.step(steps)
    o.update_derived()
    return o.rho[0, 100, 0], o.rho[0, 0, 0], float(np.abs(o.velocity()).max())


@pytest.mark.parametrize("Tr,steps,tol_l,tol_g", [(0.95, 60000, 5e-4, 1e-3), (0.8, 80000, 1e-4, 1e-2)])
def test_flat_interface_reaches_maxwell_coexistence(Tr, steps, tol_l, tol_g):
    # Sec. II B: with the force of Eq. 7 a flat interface at rest sits at the
    # Maxwell coexistence densities of the Peng-Robinson EOS, up to the
    # discretisation of a few-lattice-unit interface (smallest near Tc)
    rl, rg, umax = _relaxed_slab(Tr, steps)
    m = O.maxwell(Tr)
    assert umax < 1e-6
    assert abs(rl / m["rho_l"] - 1) < tol_l, (rl, m["rho_l"])
    assert abs(rg / m["rho_g"] - 1) < tol_g, (rg, m["rho_g"])


def test_flat_interface_gas_density_gap_at_tr_06():
    # at Tr = 0.6 (density ratio about 850) the liquid still sits within 1e-3
    # of Maxwell's value, but the gas settles near 3.5 times its value: the
    # interface is about three lattice units thick and the fourth-order
    # stencils do not resolve its gas side.  The gap is a property of the
    # discretised model, recorded here so that a change to it shows.
    rl, rg, umax = _relaxed_slab(0.6, 40000)
    m = O.maxwell(0.6)
    assert umax < 1e-3
    assert abs(rl / m["rho_l"] - 1) < 1e-3
    assert 3.0 < rg / m["rho_g"] < 4.0, rg / m["rho_g"]


# ---------------------------------------------------------------- lattice, MRT, forcing


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_isotropy(dim):
    e, w = O.lattice(dim)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose((w[:, None] * e).sum(0), 0)
    second = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(second, np.eye(3)[:, :] * (1 / 3) * (np.arange(3)[:, None] < dim) * (np.arange(3) < dim))
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    sl = slice(0, dim)
    assert np.allclose(fourth[sl, sl, sl, sl], iso[sl, sl, sl, sl])


@pytest.mark.parametrize("dim", [2, 3])
def test_mrt_basis_orthogonal(dim):
    M = O.mrt_matrix(dim)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0)
    e, w = O.lattice(dim)
    # conserved rows are density and momentum
    assert np.array_equal(M[0], np.ones(len(w)))
    mom = [3, 5] if dim == 2 else [3, 5, 7]
    for a, r in enumerate(mom):
        assert np.array_equal(M[r], e[:, a])


def test_d2q9_equilibrium_moments():
    # the Lallemand-Luo equilibria of the D2Q9 moments follow from Eq. 2
    M = O.mrt_matrix(2)
    rho, u = 1.3, np.array([0.05, -0.03])
    m = M @ O.feq(2, rho, u)
    jx, jy = rho * u
    uu = u @ u
    ref = [rho, -2 * rho + 3 * rho * uu, rho - 3 * rho * uu, jx, -jx, jy, -jy, rho * (u[0] ** 2 - u[1] ** 2),
           rho * u[0] * u[1]]
    assert np.allclose(m, ref, atol=1e-15)


def _params(dim, **kw):
    return O.make_params(dim, (8, 8, 8 if dim == 3 else 1), **kw)


@pytest.mark.parametrize("dim", [2, 3])
def test_edm_forcing_moments(dim):
    # Eq. 13 adds exactly the force: sum F_i = 0, sum F_i e_i = F (with f = f_eq
    # the relaxation term vanishes, so the collision output is f_eq + F_i)
    rng = np.random.Generator(np.random.PCG64(3))
    e, w = O.lattice(dim)
    for _ in range(5):
        rho = rng.uniform(0.5, 3.0)
        u = np.zeros(3)
        u[:dim] = rng.uniform(-0.05, 0.05, dim)
        F = np.zeros(3)
        F[:dim] = rng.uniform(-0.02, 0.02, dim)
        f = O.feq(dim, rho, u)
        out = O.collide_node(_params(dim), f, F)
        d = out - f
        assert abs(d.sum()) < 1e-15
        assert np.allclose(d @ e, F, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_mrt_equal_rates_is_bgk(dim):
    rng = np.random.Generator(np.random.PCG64(5))
    tau = 0.8
    r = 1.0 / tau
    f = O.feq(dim, 1.1, [0.02, -0.01, 0.01]) * (1 + 0.05 * rng.uniform(-1, 1, 9 if dim == 2 else 19))
    F = [0.003, -0.002, 0.001]
    mrt = O.collide_node(_params(dim, tau=tau, s_e=r, s_eps=r, s_q=r, s_pi=r, s_m=r), f, F)
    bgk = O.collide_node(_params(dim, tau=tau, bgk=1), f, F)
    # BGK by hand: f - (f - f_eq)/tau + f_eq(rho, u + F/rho) - f_eq(rho, u)
    e, w = O.lattice(dim)
    rho = f.sum()
    u = (f @ e) / rho
    ref = f - (f - O.feq(dim, rho, u)) / tau + O.feq(dim, rho, u + np.array(F) / rho) - O.feq(dim, rho, u)
    assert np.allclose(mrt, ref, atol=1e-14)
    assert np.allclose(bgk, ref, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_tau_one_bgk_gives_shifted_equilibrium(dim):
    f = O.feq(dim, 0.9, [0.01, 0.02, -0.01]) * 1.01
    F = np.array([0.001, -0.003, 0.002])
    out = O.collide_node(_params(dim, tau=1.0, bgk=1), f, F)
    e, _ = O.lattice(dim)
    rho = f.sum()
    u = (f @ e) / rho
    assert np.allclose(out, O.feq(dim, rho, u + F / rho), atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_mrt_conserves_and_relaxes(dim):
    # D2Q9 rates of Sec. II A: conserved moments unchanged, the others relaxed by s_k
    M = O.mrt_matrix(dim)
    f = O.feq(dim, 1.2, [0.03, 0.01, -0.02]) * (1 + 0.02 * np.cos(np.arange(9 if dim == 2 else 19)))
    out = O.collide_node(_params(dim), f, [0, 0, 0])
    m, mo = M @ f, M @ out
    e, _ = O.lattice(dim)
    rho = f.sum()
    meq = M @ O.feq(dim, rho, (f @ e) / rho)
    s = [0, 1.64, 1.54, 0, 1.9, 0, 1.9, 1.0, 1.0] if dim == 2 else \
        [0, 1.64, 1.54, 0, 1.9, 0, 1.9, 0, 1.9, 1.0, 1.54, 1.0, 1.54, 1.0, 1.0, 1.0, 1.9, 1.9, 1.9]
    assert np.allclose(mo, m - np.array(s) * (m - meq), atol=1e-14)


# ---------------------------------------------------------------- stencils, chemical potential, force


def _poly_field(shape, coef, deg):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return sum(c * (x - 7.3) ** p + c * 0.5 * (y - 6.1) ** p + c * 0.25 * (z - 5.2) ** p
               for p, c in zip(range(deg + 1), coef)), (x, y, z)


@pytest.mark.parametrize("dim", [2, 3])
def test_laplacian_exact_on_quintics(dim):
    # fourth-order Laplacian: exact on polynomials of degree <= 5.  With k tiny
    # the chemical potential of Eq. 12 is -kappa lap(rho) alone.
    n = (16, 14, 12 if dim == 3 else 1)
    o = O.Oracle(dim, n, wall=(1, 1, 1 if dim == 3 else 0), k=1e-30, kappa=0.5)
    coef = [5.0, 1e-2, 3e-3, 2e-4, 1e-5, 3e-7]
    rho, (x, y, z) = _poly_field(o.shape, coef, 5)
    if dim == 2:
        rho = coef[0] + sum(c * (x - 7.3) ** p + c * 0.5 * (y - 6.1) ** p for p, c in zip(range(6), coef)) - coef[0]
    o.rho[...] = rho
    o.phase("mu")
    lap = np.zeros_like(rho)
    axes = [(x - 7.3, 1.0), (y - 6.1, 0.5)] + ([(z - 5.2, 0.25)] if dim == 3 else [])
    for q, sc in axes:
        lap += sum(sc * c * p * (p - 1) * q ** (p - 2) for p, c in zip(range(2, 6), coef[2:]))
    inner = o.cls == 0
    assert np.max(np.abs(o.mu[inner] + 0.5 * lap[inner])) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_exact_on_quartics(dim):
    # F = -rho grad(mu) + cs^2 grad(rho): with rho constant, F = -rho grad(mu);
    # the fourth-order gradient is exact on quartics
    n = (16, 14, 12 if dim == 3 else 1)
    o = O.Oracle(dim, n, wall=(1, 1, 1 if dim == 3 else 0))
    nz, ny, nx = o.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mu = 0.1 + 1e-3 * (x - 3) ** 4 - 2e-3 * (y - 2) ** 3 + (4e-4 * (z - 1) ** 4 if dim == 3 else 0)
    o.rho[...] = 2.0
    o.mu[...] = mu
    o.phase("force")
    gx, gy = 4e-3 * (x - 3) ** 3, -6e-3 * (y - 2) ** 2
    inner = o.cls == 0
    F = o.force
    assert np.max(np.abs(F[0][inner] + 2.0 * gx[inner])) < 1e-12
    assert np.max(np.abs(F[1][inner] + 2.0 * gy[inner])) < 1e-12
    if dim == 3:
        gz = 1.6e-3 * (z - 1) ** 3
        assert np.max(np.abs(F[2][inner] + 2.0 * gz[inner])) < 1e-12
    # and with mu constant, F = grad(rho)/3
    o.mu[...] = 0.3
    o.rho[...] = 1.0 + 1e-2 * (x - 3) ** 2
    o.phase("force")
    assert np.max(np.abs(F[0][inner] - 2e-2 * (x - 3)[inner] / 3)) < 1e-13


def test_chemical_potential_uses_eq11():
    # with kappa = 0 the fluid chemical potential is k^2 psi'(rho)
    o = O.Oracle(2, (12, 10), k=0.3, kappa=0.0)
    rng = np.random.Generator(np.random.PCG64(1))
    o.rho[...] = rng.uniform(0.05, 8.0, o.shape)
    o.phase("mu")
    inf = o.info()
    ref = np.vectorize(lambda r: 0.09 * O.pr_mu(r, inf["T"], inf["alpha"]))(o.rho)
    assert np.allclose(o.mu, ref, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- solids, boundary


def test_fill_constant_field():
    # Eq. 14 is a weighted mean: a constant field stays constant on both layers
    o = O.Oracle(2, (40, 40), wall=(1, 0))
    o.add_sphere((20.3, 19.6), 8.4, mu_w=0.02)
    o.rho[...] = np.where(o.cls == 0, 3.25, -7.0)
    o.phase("fill")
    lay = (o.cls == 1) | (o.cls == 2)
    assert lay.sum() > 50
    assert np.all(np.abs(o.rho[lay] - 3.25) < 1e-15)


def test_layer_classes():
    o = O.Oracle(2, (40, 40))
    o.add_sphere((20.0, 20.0), 9.5)
    cls = o.cls[0]
    yy, xx = np.mgrid[0:40, 0:40]
    inside = (xx - 20.0) ** 2 + (yy - 20.0) ** 2 <= 9.5**2
    assert np.array_equal(cls == 0, ~inside)
    e, _ = O.lattice(2)
    for yv, xv in zip(*np.nonzero(inside)):
        nb = [cls[yv + ey, xv + ex] for ex, ey, _ in e[1:]]
        if 0 in nb:
            assert cls[yv, xv] == 1
        elif 1 in nb:
            assert cls[yv, xv] == 2
        else:
            assert cls[yv, xv] == 3


def test_link_fraction_closed_form():
    # axis link from (x,y) toward a circle centred on the same row: q = (x_c - R) - x... exact
    o = O.Oracle(2, (40, 40))
    o.add_sphere((20.0, 20.0), 5.3)
    # node (14, 20): distance to the wall along +x is 20 - 5.3 - 14 = 0.7
    assert abs(o.link_q(14, 20, 0, 1) - 0.7) < 1e-14
    # diagonal link from (15, 16) along (1,1): |(15,16) + q(1,1) - (20,20)| = 5.3
    q = o.link_q(15, 16, 0, 5)
    p = np.array([15 + q, 16 + q]) - 20
    assert abs(np.hypot(*p) - 5.3) < 1e-13 and 0 < q <= 1
    assert o.link_q(10, 10, 0, 1) == -1


def test_halfway_equals_interpolated_at_half():
    # box walls cut every link at q = 1/2: both wall schemes give identical states
    kw = dict(wall=(1, 1))
    a = O.Oracle(2, (30, 26), bc_mode=0, **kw)
    b = O.Oracle(2, (30, 26), bc_mode=1, **kw)
    for o in (a, b):
        o.init_drops([(15, 13)], [6], W=10)
        o.step(30)
    assert np.array_equal(a.f, b.f)


@pytest.mark.parametrize("bc", [0, 1])
def test_mass_conservation(bc):
    o = O.Oracle(2, (64, 64), bc_mode=bc, Tr=0.8)
    o.add_sphere((32.4, 20.7), 12.3, mu_w=0.05)
    o.init_drops([(32, 42)], [9], W=10)
    m0 = o.mass()
    o.step(300)
    assert abs(o.mass() / m0 - 1) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("phase", ["liquid", "gas"])
def test_uniform_state_is_fixed_point(dim, phase):
    o = O.Oracle(dim, (10, 9, 8 if dim == 3 else 1))
    inf = o.info()
    r = inf["rho_l"] if phase == "liquid" else inf["rho_g"]
    o.set_rho(np.full(o.shape, r))
    f0 = o.f.copy()
    o.step(200 if dim == 3 else 1000)
    assert np.max(np.abs(o.f - f0)) <= 1e-14 * r


def test_mirror_symmetry_2d():
    # the sessile 2-D layout is symmetric about x = 64 (node 0 is its own image)
    o = O.Oracle(2, (128, 128))
    o.add_sphere((64, 40), 24, mu_w=0.04)
    o.init_drops([(64, 84)], [20], W=10)
    o.step(300)
    r = o.rho[0]
    assert np.max(np.abs(r[:, 1:] - r[:, 1:][:, ::-1])) < 1e-11
    a = o.measure()
    assert abs(a.sector_deg[0] - a.sector_deg[1]) < 1e-7


# ---------------------------------------------------------------- measurement


@pytest.mark.parametrize("theta0", [30, 60, 90, 120, 150])
def test_wedge_drop_measured_exactly(theta0):
    # straight interfaces meeting a circle at theta0 with an affine density
    # profile: every isodensity crossing lies on the line, so the secant is the
    # line and the measured angle is theta0 (Sec. III B, Eq. 15)
    o = O.Oracle(2, (200, 180))
    o.add_sphere((100, 60), 60, mu_w=0.0)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    o.set_rho(W.wedge_density(o.shape, (100, 60), 60, theta0, rm, inf["rho_g"], inf["rho_l"]))
    a = o.measure()
    assert a.status == 0 and a.n_valid == 2
    assert abs(a.sector_deg[0] - theta0) < 1e-9
    assert abs(a.sector_deg[1] - theta0) < 1e-9
    # the contact points are the circle points at +-30 lu from the axis
    for s, sign in ((0, 1), (1, -1)):
        assert abs(a.contact[s][0] - (100 + sign * 30)) < 1e-9
        assert abs(a.contact[s][1] - (60 + 60 * math.cos(math.asin(0.5)))) < 1e-9


@pytest.mark.parametrize("mu_w", [-0.01, 0.1])
def test_relaxed_drop_agrees_with_spherical_cap(mu_w):
    # Sec. IV A: without gravity the drop relaxes to a circular cap, and the
    # spherical-cap method gives its angle from the base length L (between the
    # two contact points) and the height H above that chord: R0 = (4 H^2 +
    # L^2) / 8 H, tan(beta) = L / 2 (R0 - H), theta = beta - alpha on a convex
    # substrate, alpha the half-angle of the chord seen from the substrate
    # centre.  The in-step measurement uses only the interface within 2.5 lu of
    # the substrate; the cap method uses the whole drop.
    wl = W.sessile_2d(mu_w=mu_w)                      # 128^2, cylinder 24, drop 20, Tr = 0.6
    o = O.Oracle(2, wl["n"], (0, 0), Tr=wl["Tr"], k=0.28, kappa=0.01)
    sol = wl["solids"][0]
    o.add_sphere(sol["center"], sol["radius"], mu_w=mu_w)
    o.init_drops([c for c, _ in wl["drops"]], [r for _, r in wl["drops"]], W=10.0)
    o.step(8000)
    a = o.measure()
    assert a.status == 0 and a.n_valid == 2
    o.update_derived()
    nx, ny = wl["n"]
    rho, cls = o.rho.reshape(ny, nx), o.cls.reshape(ny, nx)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    pts = []
    for dx, dy in ((1, 0), (0, 1)):                   # rho_m crossings on fluid-fluid links
        r0, r1 = rho[: ny - dy, : nx - dx], rho[dy:, dx:]
        ok = (cls[: ny - dy, : nx - dx] == 0) & (cls[dy:, dx:] == 0) & ((r0 - rm) * (r1 - rm) < 0)
        yy, xx = np.nonzero(ok)
        t = (rm - r0[ok]) / (r1[ok] - r0[ok])
        pts.append(np.c_[xx + t * dx, yy + t * dy])
    pts = np.vstack(pts)
    cs, Rs = np.array(sol["center"][:2]), sol["radius"]
    c1, c2 = np.array(a.contact[0][:2]), np.array(a.contact[1][:2])
    L = np.linalg.norm(c2 - c1)
    mid = 0.5 * (c1 + c2)
    up = (mid - cs) / np.linalg.norm(mid - cs)
    H = float(np.max((pts - mid) @ up))
    R0 = (4 * H * H + L * L) / (8 * H)
    beta = math.degrees(math.atan2(L, 2 * (R0 - H)))
    alpha = math.degrees(math.asin(0.5 * L / Rs))
    assert abs(a.mean_deg - (beta - alpha)) < 1.5, (a.mean_deg, beta - alpha)


def test_no_liquid_no_contact_line():
    o = O.Oracle(2, (40, 40))
    o.add_sphere((20, 10), 6, mu_w=0.0)
    o.set_rho(np.full(o.shape, o.info()["rho_g"]))
    a = o.measure()
    assert a.status == -6 and math.isnan(a.mean_deg)


# ------------------------------------------------------------ Laplace's law


def _bulk_roots(mu_hat, T, alpha, k):
    """Gas and liquid densities whose bulk chemical potential k^2 psi'(rho) is mu_hat."""
    from scipy.optimize import brentq
    g = lambda r: k * k * O.pr_mu(r, T, alpha) - mu_hat  # noqa: E731
    grid = np.linspace(1e-3, 1.0 / O.PR_B - 1e-3, 4000)
    vals = np.array([g(r) for r in grid])
    idx = np.nonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    assert len(idx) == 3, "chemical potential outside the two-phase window"
    return (brentq(g, grid[idx[0]], grid[idx[0] + 1], xtol=1e-15),
            brentq(g, grid[idx[-1]], grid[idx[-1] + 1], xtol=1e-15))


def test_laplace_law_free_drops():
    """Laplace's law for a free drop (2-D: Delta p = gamma / R).

    Drops of three radii relax in periodic boxes.  At equilibrium the
    chemical potential is uniform (the force of Eq. 7 vanishes where mu is
    constant; on the lattice up to about a tenth of its rise mu - mu_sat, so
    the mean of the liquid and gas values is used); the pressure jump follows from the Peng-Robinson bulk pressures
    of the liquid and the gas that have that chemical potential (Gibbs-Duhem),
    and R is the equimolar radius.  Laplace's law holds if R Delta p, the
    surface tension, is the same for every drop.
    """
    Tr, k, kappa = 0.8, 0.28, 0.01
    mx = O.maxwell(Tr)
    T, al = mx["T"], mx["alpha"]
    gam = []
    for R, n in ((12, 64), (16, 72), (24, 96)):
        o = O.Oracle(2, (n, n), (0, 0), Tr=Tr, k=k, kappa=kappa)
        o.init_drops([(n / 2, n / 2)], [R], W=10.0)
        o.step(4000)
        o.update_derived()
        rho, mu = o.rho.reshape(n, n), o.mu.reshape(n, n)
        mu_in, mu_out = mu[n // 2, n // 2], mu[0, 0]
        dmu = 0.5 * (mu_in + mu_out) - k * k * mx["mu_sat"]
        # raised by the curvature, and uniform up to the discretisation's residual
        assert dmu > 0 and abs(mu_in - mu_out) < 0.15 * dmu
        rg, rl = _bulk_roots(0.5 * (mu_in + mu_out), T, al, k)
        assert abs(rho[0, 0] / rg - 1) < 0.02 and abs(rho[n // 2, n // 2] / rl - 1) < 0.02
        dp = k * k * (O.pr_p0(rl, T, al) - O.pr_p0(rg, T, al))
        Re = math.sqrt(((rho - rg) / (rl - rg)).sum() / math.pi)
        assert abs(Re / R - 1) < 0.1
        gam.append(dp * Re)
    assert max(gam) / min(gam) - 1 < 0.04, gam


# ------------------------------------------------------ brute force on 8 x 8


def test_one_step_matches_brute_force_on_8x8():
    """One whole step of a periodic 8 x 8 D2Q9 lattice without solids, computed
    by brute force with array shifts: rho, the chemical potential of Eq. 12
    (fourth-order Laplacian), the force of Eq. 7 (fourth-order gradients), the
    MRT collision of Eq. 1 in the moment basis built from its polynomials, the
    exact-difference forcing of Eq. 13, and the streaming of Eq. 4."""
    Tr, k, kappa, tau, s_e, s_eps, s_q = 0.8, 0.28, 0.01, 1.0, 1.64, 1.54, 1.9
    o = O.Oracle(2, (8, 8), Tr=Tr, k=k, kappa=kappa, tau=tau, s_e=s_e, s_eps=s_eps, s_q=s_q)
    rng = np.random.Generator(np.random.PCG64(8))
    o.set_rho(rng.uniform(0.3, 6.5, o.shape))
    o.step(1)                                     # a state with non-equilibrium parts
    f = o.f.copy()[:, 0]                          # [Q][y][x]
    inf = o.info()
    e, w = O.lattice(2)
    ex, ey = e[:, 0].astype(float), e[:, 1].astype(float)

    def sh(a, dx, dy):                            # a(x + dx, y + dy), periodic
        return np.roll(np.roll(a, -dy, axis=0), -dx, axis=1)

    def d1(a, ax):
        s = (lambda j: sh(a, j, 0)) if ax == 0 else (lambda j: sh(a, 0, j))
        return (s(-2) - 8 * s(-1) + 8 * s(1) - s(2)) / 12.0

    def lap(a):
        return sum((-sh(a, 2 * dx, 2 * dy) + 16 * sh(a, dx, dy) - 30 * a + 16 * sh(a, -dx, -dy)
                    - sh(a, -2 * dx, -2 * dy)) / 12.0 for dx, dy in ((1, 0), (0, 1)))

    rho = f.sum(0)
    psi1 = np.vectorize(lambda r: O.pr_mu(r, inf["T"], inf["alpha"]))(rho)
    mu = k * k * psi1 - kappa * lap(rho)
    Fx = -rho * d1(mu, 0) + d1(rho, 0) / 3.0
    Fy = -rho * d1(mu, 1) + d1(rho, 1) / 3.0
    ux = np.tensordot(ex, f, 1) / rho
    uy = np.tensordot(ey, f, 1) / rho

    def feq(vx, vy):
        eu = ex[:, None, None] * vx + ey[:, None, None] * vy
        return w[:, None, None] * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (vx ** 2 + vy ** 2))

    c2 = ex ** 2 + ey ** 2
    M = np.array([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 ** 2, ex, (-5 + 3 * c2) * ex,
                  ey, (-5 + 3 * c2) * ey, ex ** 2 - ey ** 2, ex * ey])
    S = np.diag([0, s_e, s_eps, 0, s_q, 0, s_q, 1 / tau, 1 / tau])
    f0, f1 = feq(ux, uy), feq(ux + Fx / rho, uy + Fy / rho)
    m, meq = np.tensordot(M, f, 1), np.tensordot(M, f0, 1)
    post = np.tensordot(np.linalg.inv(M), m - np.tensordot(S, m - meq, 1), 1) + f1 - f0
    new = np.array([sh(post[i], -int(ex[i]), -int(ey[i])) for i in range(9)])   # f_i(x) = f*_i(x - e_i)
    o.step(1)
    assert np.max(np.abs(o.f[:, 0] - new)) < 1e-13 * np.max(np.abs(new))


# ------------------------------ brute force with walls and a curved solid


def _brute_lattice(dim):
    """D2Q9 / D3Q19 from their definition: every e in {-1, 0, 1}^dim with
    |e|^2 <= 2, weights 4/9, 1/9, 1/36 (2-D) and 1/3, 1/18, 1/36 (3-D) by
    |e|^2; returned in the oracle's direction order (checked against it)."""
    import itertools
    es = [e for e in itertools.product((-1, 0, 1), repeat=dim) if sum(c * c for c in e) <= 2]
    wt = {2: (4 / 9, 1 / 9, 1 / 36), 3: (1 / 3, 1 / 18, 1 / 36)}[dim]
    eo, wo = O.lattice(dim)
    assert len(es) == len(eo)
    order = [es.index(tuple(int(v) for v in eo[i][:dim])) for i in range(len(eo))]
    e = np.array([list(es[k]) + [0] * (3 - dim) for k in order], dtype=np.int64)
    w = np.array([wt[sum(c * c for c in es[k])] for k in order])
    assert np.array_equal(e, np.asarray(eo, dtype=np.int64)) and np.allclose(w, wo, rtol=0, atol=1e-16)
    return e, w


def _brute_moments(dim, tau, s_e, s_eps, s_q, s_pi=None, s_m=None):
    """Moment rows as velocity polynomials with their rates: Lallemand-Luo for
    D2Q9, d'Humieres et al. for D3Q19 (conserved moments at rate 0, the shear
    stresses at 1 / tau)."""
    sv = 1.0 / tau
    if dim == 2:
        return [(lambda x, y, z, c2: 1.0, 0), (lambda x, y, z, c2: -4 + 3 * c2, s_e),
                (lambda x, y, z, c2: 4 - 10.5 * c2 + 4.5 * c2 * c2, s_eps), (lambda x, y, z, c2: x, 0),
                (lambda x, y, z, c2: (-5 + 3 * c2) * x, s_q), (lambda x, y, z, c2: y, 0),
                (lambda x, y, z, c2: (-5 + 3 * c2) * y, s_q), (lambda x, y, z, c2: x * x - y * y, sv),
                (lambda x, y, z, c2: x * y, sv)]
    return [(lambda x, y, z, c2: 1.0, 0), (lambda x, y, z, c2: 19 * c2 - 30, s_e),
            (lambda x, y, z, c2: (21 * c2 * c2 - 53 * c2 + 24) / 2, s_eps),
            (lambda x, y, z, c2: x, 0), (lambda x, y, z, c2: (5 * c2 - 9) * x, s_q),
            (lambda x, y, z, c2: y, 0), (lambda x, y, z, c2: (5 * c2 - 9) * y, s_q),
            (lambda x, y, z, c2: z, 0), (lambda x, y, z, c2: (5 * c2 - 9) * z, s_q),
            (lambda x, y, z, c2: 3 * x * x - c2, sv), (lambda x, y, z, c2: (3 * c2 - 5) * (3 * x * x - c2), s_pi),
            (lambda x, y, z, c2: y * y - z * z, sv), (lambda x, y, z, c2: (3 * c2 - 5) * (y * y - z * z), s_pi),
            (lambda x, y, z, c2: x * y, sv), (lambda x, y, z, c2: y * z, sv), (lambda x, y, z, c2: x * z, sv),
            (lambda x, y, z, c2: (y * y - z * z) * x, s_m), (lambda x, y, z, c2: (z * z - x * x) * y, s_m),
            (lambda x, y, z, c2: (x * x - y * y) * z, s_m)]


def _brute_step(dim, n, wall, f, prm, discs, wall_mu, bc):
    """One whole step by the definitions, node by node: classes of Sec. III A
    (solid = a disc/ball or the two outer layers of a wall axis; first layer =
    solid with a fluid neighbour, second = solid with a first-layer one), the
    fill of Eq. 14 (w-weighted mean of the fluid neighbours, then of the
    first-layer ones), the chemical potential of Eq. 11 on fluid nodes and the
    prescribed one on both layers, the force of Eq. 7 with gravity, the MRT
    collision of Eq. 1 with the forcing of Eq. 13, and the pull streaming of
    Eq. 4 with the missing populations from halfway bounce-back (bc 0) or
    Bouzidi's linear interpolation (bc 1; q the root of |x + q e - C| = R
    found by bisection, 1/2 at a wall), the difference to the bounced-back
    population going to the rest population.  f is [Q][z][y][x]."""
    from scipy.optimize import brentq
    e, w = _brute_lattice(dim)
    Q = len(w)
    opp = [int(np.nonzero((e == -e[i]).all(1))[0][0]) for i in range(Q)]
    nx, ny, nz = (list(n) + [1])[:3]
    size = (nx, ny, nz)

    def wrap(p):
        # periodic axes wrap; a wall axis never needs to (two solid layers)
        q = list(p)
        for d in range(dim):
            if q[d] < 0 or q[d] >= size[d]:
                if wall[d]:
                    return None
                q[d] %= size[d]
        return tuple(q)

    def in_disc(p):
        for c, r, muw in discs:
            if sum((p[d] - c[d]) ** 2 for d in range(dim)) <= r * r:
                return (c, r, muw)
        return None

    def in_wall(p):
        return any(wall[d] and (p[d] < 2 or p[d] >= size[d] - 2) for d in range(dim))

    nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    solid = {p: bool(in_disc(p) or in_wall(p)) for p in nodes}
    nbrs = {p: [wrap((p[0] + e[i][0], p[1] + e[i][1], p[2] + e[i][2])) for i in range(Q)] for p in nodes}
    cls = {}
    for p in nodes:
        cls[p] = 0 if not solid[p] else (1 if any(m and not solid[m] for m in nbrs[p][1:]) else 3)
    for p in nodes:
        if cls[p] == 3 and any(m and cls[m] == 1 for m in nbrs[p][1:]):
            cls[p] = 2
    fx = {p: f[:, p[2], p[1], p[0]] for p in nodes}
    rho = {p: fx[p].sum() if cls[p] == 0 else 0.0 for p in nodes}
    for layer, src in ((1, 0), (2, 1)):
        for p in nodes:
            if cls[p] == layer:
                ws = [(w[i], rho[m]) for i, m in enumerate(nbrs[p]) if i and m and cls[m] == src]
                rho[p] = sum(a * b for a, b in ws) / sum(a for a, _ in ws)

    def shift(p, ax, k):
        q = list(p)
        q[ax] += k
        return wrap(tuple(q))

    def d1(fld, p, ax):
        v = [fld[shift(p, ax, k)] for k in (-2, -1, 1, 2)]
        return (v[0] - 8 * v[1] + 8 * v[2] - v[3]) / 12.0

    def d2(fld, p, ax):
        v = [fld[shift(p, ax, k)] for k in (-2, -1, 0, 1, 2)]
        return (-v[0] + 16 * v[1] - 30 * v[2] + 16 * v[3] - v[4]) / 12.0

    k, kappa, T, al = prm["k"], prm["kappa"], prm["T"], prm["alpha"]
    mu = {}
    for p in nodes:
        if cls[p] == 0:
            mu[p] = k * k * O.pr_mu(rho[p], T, al) - kappa * sum(d2(rho, p, ax) for ax in range(dim))
        elif cls[p] in (1, 2):
            dsc = in_disc(p)
            mu[p] = dsc[2] if dsc else wall_mu
        else:
            mu[p] = 0.0
    rows = _brute_moments(dim, prm["tau"], prm["s_e"], prm["s_eps"], prm["s_q"], prm.get("s_pi"), prm.get("s_m"))
    c2 = (e * e).sum(1)
    M = np.array([[fn(*e[i], c2[i]) for i in range(Q)] for fn, _ in rows], dtype=np.float64)
    S = np.diag([r for _, r in rows])
    A = np.linalg.solve(M, S @ M)                          # M^-1 S M
    g = np.array(prm["g"], dtype=np.float64)

    def feq(r, u):
        eu = e @ u
        return w * r * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (u @ u))

    post = {}
    for p in nodes:
        if cls[p] != 0:
            post[p] = np.zeros(Q)
            continue
        r = rho[p]
        F = np.zeros(3)
        for ax in range(dim):
            F[ax] = -r * d1(mu, p, ax) + d1(rho, p, ax) / 3.0 + r * g[ax]
        u = (e.T @ fx[p]) / r
        f0, f1 = feq(r, u), feq(r, u + F / r)
        post[p] = fx[p] - A @ (fx[p] - f0) + f1 - f0

    def link_q(p, j):
        t = nbrs[p][j]
        if in_wall(t):
            return 0.5
        c, rr, _ = in_disc(t)
        dist = lambda s: math.sqrt(sum((p[d] + s * e[j][d] - c[d]) ** 2 for d in range(dim))) - rr  # noqa: E731
        return brentq(dist, 0.0, 1.0, xtol=1e-15, rtol=1e-15)

    out = np.zeros_like(f)
    used_q, kept_q = [], []    # links interpolated; links with q < 1/2 left halfway (partner of the other phase)
    for p in nodes:
        if cls[p] != 0:
            continue
        new = np.zeros(Q)
        dm = 0.0
        for i in range(1, Q):
            src = wrap((p[0] - e[i][0], p[1] - e[i][1], p[2] - e[i][2]))
            if cls[src] == 0:
                new[i] = post[src][i]
                continue
            j = opp[i]
            back = post[p][j]
            val = back
            if bc == 1:
                q = link_q(p, j)
                xb = nbrs[p][i]
                if q < 0.5 and cls[xb] == 0:
                    # interpolation only between two populations of direction j
                    # that lie within a factor of two of each other
                    fb = post[xb][j]
                    if fb <= 2 * back and back <= 2 * fb:
                        val = 2 * q * back + (1 - 2 * q) * fb
                        used_q.append(q)
                    else:
                        kept_q.append(q)
                elif q >= 0.5:
                    val = back / (2 * q) + (2 * q - 1) / (2 * q) * post[p][i]
                    used_q.append(q)
            new[i] = val
            dm += back - val
        new[0] = post[p][0] + dm
        out[:, p[2], p[1], p[0]] = new
    return out, cls, (used_q, kept_q)


@pytest.mark.parametrize("bc", [0, 1])
def test_one_step_with_walls_and_a_disc_matches_brute_force(bc):
    """16 x 16 D2Q9: walls on y (two solid layers each side, their own wall
    chemical potential), periodic x, an off-node disc of radius 3.4 with its
    own, tilted gravity, and a non-uniform state with non-equilibrium parts;
    one oracle step equals the brute-force step above to 1e-12, with the
    interpolated wall using links on both sides of q = 1/2, and links with
    q < 1/2 whose partner population differs by more than a factor of two
    (the random density field spans a factor of five) left at the halfway value."""
    prm = dict(Tr=0.8, k=0.28, kappa=0.01, tau=0.8, s_e=1.64, s_eps=1.54, s_q=1.9, g=(3e-4, -2e-4, 0.0))
    o = O.Oracle(2, (16, 16), (0, 1), bc_mode=bc, wall_mu=0.021, **prm)
    disc = ((7.3, 8.6), 3.4, 0.057)
    o.add_sphere(disc[0], disc[1], mu_w=disc[2])
    rng = np.random.Generator(np.random.PCG64(16))
    o.set_rho(rng.uniform(1.0, 5.0, o.shape))
    o.step(1)                                        # a state with non-equilibrium parts
    f = o.f.copy()
    inf = o.info()
    prm.update(T=inf["T"], alpha=inf["alpha"])
    new, cls, used = _brute_step(2, (16, 16), (0, 1), f, prm, [disc], 0.021, bc)
    assert all(o.cls[0, y, x] == cls[(x, y, 0)] for y in range(16) for x in range(16))
    assert {1, 2} <= set(cls.values())
    if bc == 1:
        used, kept = used
        assert min(used) < 0.35 and max(used) > 0.65 and any(abs(q - 0.5) < 1e-15 for q in used), sorted(used)
        assert any(q < 0.5 for q in used) and kept, (sorted(used), sorted(kept))
    o.step(1)
    assert np.max(np.abs(o.f - new)) < 1e-12 * np.max(np.abs(new))
    # the fluid mass is what it was (the mass correction of the interpolated wall)
    assert abs(new.sum() / f.sum() - 1) < 1e-13


def test_one_step_d3q19_matches_brute_force_on_8x8x8():
    """8 x 8 x 8 D3Q19, periodic x and y, walls on z (four fluid planes), MRT
    with five distinct rates in the d'Humieres basis, gravity in all three
    directions: one oracle step equals the brute-force step to 1e-12."""
    prm = dict(Tr=0.8, k=0.28, kappa=0.01, tau=0.8, s_e=1.64, s_eps=1.54, s_q=1.9, s_pi=1.3, s_m=1.7,
               g=(2e-4, -1e-4, -3e-4))
    o = O.Oracle(3, (8, 8, 8), (0, 0, 1), wall_mu=0.03, **prm)
    rng = np.random.Generator(np.random.PCG64(8))
    o.set_rho(rng.uniform(1.0, 5.0, o.shape))
    o.step(1)
    f = o.f.copy()
    inf = o.info()
    prm.update(T=inf["T"], alpha=inf["alpha"])
    new, cls, _ = _brute_step(3, (8, 8, 8), (0, 0, 1), f, prm, [], 0.03, 0)
    assert all(o.cls[z, y, x] == cls[(x, y, z)] for z in range(8) for y in range(8) for x in range(8))
    o.step(1)
    assert np.max(np.abs(o.f - new)) < 1e-12 * np.max(np.abs(new))


# --------------------------------------------- unbalanced Young force (Eq. 17, 18)


def _wedge_on(theta0, stripes=None, slope=1.0):
    # the wedge drop of the exact-measurement pin on a uniform or striped circle
    o = O.Oracle(2, (200, 180))
    o.add_sphere((100, 60), 60, mu_w=0.0, stripes=stripes)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    o.set_rho(W.wedge_density(o.shape, (100, 60), 60, theta0, rm, inf["rho_g"], inf["rho_l"], slope=slope))
    return o


@pytest.mark.parametrize("theta0", [60, 120])
def test_young_force_on_a_uniform_surface(theta0):
    # one surface: phi_d = 1, theta_eq = theta_s1 (Eq. 18 with phi_d = 1, r = 1)
    # and F = gamma (cos theta - cos theta_s1) (Eq. 17), theta the measured angle
    o = _wedge_on(theta0)
    a, y = o.young_force(gamma=0.07, theta1_deg=100.0, theta2_deg=40.0)
    assert a.status == 0 and y.status == 0 and a.n_valid == 2
    for s in range(2):
        assert y.count[s][0] > 0 and y.count[s][1] == 0
        assert y.phi_d[s] == 1.0
        assert abs(y.theta_eq_deg[s] - 100.0) < 1e-12
        ref = 0.07 * (math.cos(math.radians(theta0)) - math.cos(math.radians(100.0)))
        assert abs(y.force[s] - ref) < 1e-12
    assert y.count[0][0] == y.count[1][0]        # mirror-symmetric footprints


def test_young_force_on_the_second_stripe():
    # the contact points sit at polar angle 30 deg on the circle of radius 60
    # (arc length 31.4 from the pole); with stripes 20 wide they lie on stripe
    # 1 (mu_w2), 11 lu from either border, and so does the whole footprint:
    # phi_d = 0, theta_eq = theta_s2
    o = _wedge_on(90, stripes=(0.0, 0.05, 20.0))
    a, y = o.young_force(gamma=0.05, theta1_deg=70.0, theta2_deg=130.0)
    assert a.status == 0
    for s in range(2):
        assert y.count[s][0] == 0 and y.count[s][1] > 0
        assert y.phi_d[s] == 0.0 and abs(y.theta_eq_deg[s] - 130.0) < 1e-12
        ref = 0.05 * (math.cos(math.radians(a.sector_deg[s])) - math.cos(math.radians(130.0)))
        assert abs(y.force[s] - ref) < 1e-12


def test_young_force_at_a_stripe_border():
    # a border that crosses the footprint splits it (Eq. 18): phi_d strictly
    # between 0 and 1, and growing as the border moves away from the pole
    # (more of the footprint on the first stripe); both sides alike by symmetry
    arc = 60 * math.pi / 6                           # arc length of the contact points
    phis = []
    for width in (arc - 1.0, arc, arc + 1.0):
        o = _wedge_on(90, stripes=(0.0, 0.05, width))
        a, y = o.young_force(gamma=0.05, theta1_deg=70.0, theta2_deg=130.0)
        assert y.count[0][0] == y.count[1][0] and y.count[0][1] == y.count[1][1]
        assert 0.0 < y.phi_d[0] < 1.0
        c = y.phi_d[0] * math.cos(math.radians(70.0)) + (1 - y.phi_d[0]) * math.cos(math.radians(130.0))
        assert abs(math.cos(math.radians(y.theta_eq_deg[0])) - c) < 1e-12
        phis.append(y.phi_d[0])
    assert phis[0] < phis[1] < phis[2]


# ------------------------------------------------ concave substrate (Fig. 2b)


def test_cavity_classes_and_link_fractions():
    # a cavity is the complement of a ball: the fluid is the open disc, the
    # first solid layer is every solid node with a fluid lattice neighbour and
    # the second every other solid node next to the first
    o = O.Oracle(2, (40, 40))
    o.add_sphere((20.0, 20.0), 9.5, cavity=True)
    cls = o.cls[0]
    yy, xx = np.mgrid[0:40, 0:40]
    fluid = (xx - 20.0) ** 2 + (yy - 20.0) ** 2 < 9.5**2
    assert np.array_equal(cls == 0, fluid)
    e, _ = O.lattice(2)
    for yv, xv in zip(*np.nonzero(~fluid)):
        nb = [cls[(yv + ey) % 40, (xv + ex) % 40] for ex, ey, _ in e[1:]]
        assert cls[yv, xv] == (1 if 0 in nb else 2 if 1 in nb else 3)
    # cut links end on the circle, seen from inside: along +x from (25, 20)
    # the wall of radius 5.3 is 0.3 away; along (1, 1) from (23, 23) it is
    # where (3 + q) sqrt(2) = 5.3
    o = O.Oracle(2, (40, 40))
    o.add_sphere((20.0, 20.0), 5.3, cavity=True)
    assert abs(o.link_q(25, 20, 0, 1) - 0.3) < 1e-14
    q = o.link_q(23, 23, 0, 5)
    assert abs(q - (5.3 / math.sqrt(2.0) - 3.0)) < 1e-14 and 0 < q <= 1
    assert o.link_q(20, 20, 0, 1) == -1


@pytest.mark.parametrize("theta0", [30, 60, 90, 120, 150])
def test_cavity_wedge_measured_exactly(theta0):
    # a pool at the bottom of a cavity of radius 80 whose straight sides meet
    # the wall at theta0: the substrate normal now points toward the centre,
    # and the measured angle is theta0 to round-off on both sides
    o = O.Oracle(2, (200, 180))
    o.add_sphere((100, 90), 80, mu_w=0.0, cavity=True)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    o.set_rho(W.cavity_wedge_density(o.shape, (100, 90), 80, theta0, rm, inf["rho_g"], inf["rho_l"]))
    a = o.measure()
    assert a.status == 0 and a.n_valid == 2
    assert list(a.axis[:2]) == [0.0, -1.0]
    for s, sign in ((0, 1), (1, -1)):
        assert abs(a.sector_deg[s] - theta0) < 1e-9
        # the contact points are the wall points 30 lu either side of the axis
        assert abs(a.contact[s][0] - (100 + sign * 30)) < 1e-9
        assert abs(a.contact[s][1] - (90 - 80 * math.cos(math.asin(30 / 80)))) < 1e-9


# ------------------------------------------ 3-D measurement (Sec. III B, Eq. 15)

SPHERE3 = ((31.5, 31.5, 26.0), 18.0)       # convex: liquid film above a plane cutting the sphere
CAVITY3 = ((31.5, 31.5, 32.0), 26.0)       # concave: pool below a plane inside a spherical cavity


def _film_on_sphere(phi_deg, cavity=False, g=(0.0, 0.0, 0.0), heights=None):
    """A 64^3 periodic lattice holding a sphere (or a cavity) and liquid bounded
    by a horizontal plane that meets it at polar angle phi from the +z pole
    (from the -z pole in the cavity).  The density is affine in z near the
    plane, so each isodensity crossing on a lattice link lies on the plane,
    and every meridional secant of Eq. 15 is exactly the plane's trace."""
    (c, r) = CAVITY3 if cavity else SPHERE3
    o = O.Oracle(3, (64, 64, 64), g=g)
    o.add_sphere(c, r, mu_w=0.0, cavity=cavity)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    if heights is None:
        h = c[2] - r * math.cos(math.radians(phi_deg)) if cavity else c[2] + r * math.cos(math.radians(phi_deg))
        heights = (h, h)
    # the far face of the liquid layer stays clear of the substrate
    far = 100.0 if cavity else 60.0 - max(heights)
    o.set_rho(W.plane_film_density(o.shape, rm, inf["rho_g"], inf["rho_l"], heights, c[0],
                                   liquid_above=not cavity, far=far))
    return o


@pytest.mark.parametrize("ns", [8, 32, 64])
@pytest.mark.parametrize("phi", [60, 90, 120])
def test_3d_plane_on_sphere_measured_exactly(phi, ns):
    # liquid above the plane z = z_c + R cos(phi): in every meridional plane
    # the liquid side of the interface is the +z half-line, the outward normal
    # at the contact point makes the angle phi with +z, so the angle through
    # the liquid is 180 - phi in every sector
    o = _film_on_sphere(phi)
    a = o.measure(0, ns)
    assert a.status == 0 and a.n_valid == ns
    assert list(a.axis) == [0.0, 0.0, 1.0]
    (c, r) = SPHERE3
    h = c[2] + r * math.cos(math.radians(phi))
    rho_c = r * math.sin(math.radians(phi))
    for s in range(ns):
        assert abs(a.sector_deg[s] - (180.0 - phi)) < 1e-9, (s, a.sector_deg[s])
        # the contact point lies on the circle where the plane cuts the sphere
        p = a.contact[s]
        assert abs(p[2] - h) < 1e-9
        assert abs(math.hypot(p[0] - c[0], p[1] - c[1]) - rho_c) < 1e-9
    assert abs(a.mean_deg - (180.0 - phi)) < 1e-9


@pytest.mark.parametrize("ns", [8, 32, 64])
@pytest.mark.parametrize("psi", [60, 90, 120])
def test_3d_pool_in_spherical_cavity_measured_exactly(psi, ns):
    # a pool at the bottom of a spherical cavity, its free surface at polar
    # angle psi from the -z pole: the substrate normal points to the centre
    # and the angle through the liquid is psi itself
    o = _film_on_sphere(psi, cavity=True)
    a = o.measure(0, ns)
    assert a.status == 0 and a.n_valid == ns
    assert list(a.axis) == [0.0, 0.0, -1.0]
    (c, r) = CAVITY3
    for s in range(ns):
        assert abs(a.sector_deg[s] - psi) < 1e-9, (s, a.sector_deg[s])
        p = a.contact[s]
        assert abs(p[2] - (c[2] - r * math.cos(math.radians(psi)))) < 1e-9
        assert abs(math.hypot(p[0] - c[0], p[1] - c[1]) - r * math.sin(math.radians(psi))) < 1e-9


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("phi", [60, 90, 120])
def test_3d_oblique_axis_measured_exactly(phi, sign):
    # the same construction about the body diagonal a = +-(1,1,1)/sqrt(3) of a
    # 72^3 lattice, with the liquid closed off by a ball of radius 33: the
    # lattice maps onto itself under the 120-degree turns about a, so the
    # centroid axis is a to round-off, and the sectors (which no longer line
    # up with lattice planes) still measure 180 - phi exactly
    n, c, r = 72, 35.5, 16.0
    a = sign * np.ones(3) / math.sqrt(3.0)
    o = O.Oracle(3, (n, n, n))
    o.add_sphere((c, c, c), r, mu_w=0.0)
    inf = o.info()
    rm = 0.5 * (inf["rho_l"] + inf["rho_g"])
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    p = np.stack([xx - c, yy - c, zz - c], -1).astype(np.float64)
    s = np.minimum(p @ a - r * math.cos(math.radians(phi)), 33.0 - np.linalg.norm(p, axis=-1))
    o.set_rho(np.clip(rm + 0.5 * s, inf["rho_g"], inf["rho_l"]))
    for ns in (8, 32):
        m = o.measure(0, ns)
        assert m.status == 0 and m.n_valid == ns
        assert np.linalg.norm(np.array(m.axis) - a) < 1e-12
        assert max(abs(t - (180.0 - phi)) for t in m.sector_deg[:ns]) < 1e-9


@pytest.mark.parametrize("tilt", [1, -1])
def test_3d_advancing_and_receding_follow_gravity(tilt):
    # a film at two heights: on the +x side of the sphere it meets it at
    # phi = 110 (angle 70), on the -x side at phi = 70 (angle 110), with a
    # six-lattice-unit ramp between them over the sphere's top.  Gravity
    # tilted 20 degrees from -z toward +x (tilt 1) makes +x the advancing
    # side.  The liquid's centroid axis leans 0.55 degrees off z, which the
    # sector angles carry as an error below 0.1 degrees at 32 and 64 sectors.
    # Turning gravity toward -x swaps the two (the selection follows g, not
    # the geometry).
    (c, r) = SPHERE3
    hl, hr = c[2] + r * math.cos(math.radians(70)), c[2] + r * math.cos(math.radians(110))
    t = math.radians(20.0)
    o = _film_on_sphere(None, g=(tilt * 1e-5 * math.sin(t), 0.0, -1e-5 * math.cos(t)), heights=(hl, hr))
    for ns in (32, 64):
        a = o.measure(0, ns)
        assert a.status == 0 and a.n_valid == ns
        adv, rec = (70.0, 110.0) if tilt > 0 else (110.0, 70.0)
        assert abs(a.adv_deg - adv) < 0.1 and abs(a.rec_deg - rec) < 0.1, (ns, a.adv_deg, a.rec_deg)
    # with gravity along the axis there is no advancing side
    o = _film_on_sphere(90)
    assert math.isnan(o.measure(0, 32).adv_deg)


def _sector_frame(a):
    # the documented sector frame: b1 = the lattice axis least aligned with a
    # (on a 1/1024 grid, ties to the lower axis), orthogonalised; b2 = a x b1
    k = min(range(3), key=lambda d: (round(abs(a[d]) * 1024), d))
    b1 = np.eye(3)[k] - a[k] * a
    b1 /= np.linalg.norm(b1)
    return b1, np.cross(a, b1)


@pytest.mark.parametrize("psi_g", [30.0, -100.0, 150.0])
def test_3d_sector_numbering_and_advancing_index(psi_g):
    # the two-height film, with gravity's tangential part at azimuth psi_g:
    # every sector's selected crossing lies in its own azimuth range, and
    # adv / rec are (bit for bit) the sectors holding psi_g and psi_g + 180
    (c, r) = SPHERE3
    hl, hr = c[2] + r * math.cos(math.radians(70)), c[2] + r * math.cos(math.radians(110))
    t, pg = math.radians(20.0), math.radians(psi_g)
    g = np.array([1e-5 * math.sin(t) * math.cos(pg), 1e-5 * math.sin(t) * math.sin(pg), -1e-5 * math.cos(t)])
    o = _film_on_sphere(None, g=tuple(g), heights=(hl, hr))
    for ns in (16, 32, 64):
        m = o.measure(0, ns)
        assert m.status == 0 and m.n_valid == ns
        a = np.array(m.axis)
        b1, b2 = _sector_frame(a)

        def sector(v):
            psi = math.atan2(v @ b2, v @ b1)
            return min(int(math.floor((psi + math.pi) / (2 * math.pi) * ns)), ns - 1)

        def in_sector(v, s):
            # a point on a sector border (here crossings on the lattice line
            # through the centre) may fall either side at round-off
            psi = math.atan2(v @ b2, v @ b1)
            lo = -math.pi + 2 * math.pi * s / ns
            hi = lo + 2 * math.pi / ns
            near = lambda x, y: abs(math.remainder(x - y, 2 * math.pi)) < 1e-12  # noqa: E731
            return sector(v) == s or near(psi, lo) or near(psi, hi)

        for s in range(ns):
            assert in_sector(np.array(m.p1[s]) - np.array(c), s)
            assert in_sector(np.array(m.p2[s]) - np.array(c), s)
        gt = g - (g @ a) * a
        sa = sector(gt)
        sr = (sa + ns // 2) % ns
        assert m.adv_deg == m.sector_deg[sa] and m.rec_deg == m.sector_deg[sr]
        # the neighbouring sectors read other angles, so an index one off would show
        for s0 in (sa, sr):
            v = m.sector_deg[s0]
            assert v != m.sector_deg[(s0 + 1) % ns] and v != m.sector_deg[(s0 - 1) % ns]


@pytest.mark.parametrize("bc", [0, 1])
def test_cavity_mass_and_mirror_symmetry(bc):
    # a drop at the bottom of a cavity, symmetric about x = 64: mass is
    # conserved to round-off and the two sides stay mirror images (Tr = 0.8:
    # the interpolated wall scheme is unstable at Tr = 0.6 on either kind of
    # substrate)
    wl = W.cavity_2d(mu_w=0.04)
    o = O.Oracle(2, wl["n"], bc_mode=bc, Tr=0.8)
    s = wl["solids"][0]
    o.add_sphere(s["center"], s["radius"], mu_w=s["mu_w"], cavity=True)
    o.init_drops([c for c, _ in wl["drops"]], [r for _, r in wl["drops"]], W=10.0)
    m0 = o.mass()
    o.step(300)
    assert abs(o.mass() / m0 - 1) < 1e-13
    r = o.rho[0]
    assert np.max(np.abs(r[:, 1:] - r[:, 1:][:, ::-1])) < 1e-11
    a = o.measure()
    assert a.status == 0 and abs(a.sector_deg[0] - a.sector_deg[1]) < 1e-7


def test_cavity_angle_grows_with_wall_potential():
    # Sec. IV A: the angle rises with the wall chemical potential, from below
    # to above 90 deg across the paper's three values (-0.01, 0.04, 0.1)
    th = []
    for mu_w in W.MU_W_SWEEP:
        wl = W.cavity_2d(mu_w=mu_w)
        o = O.Oracle(2, wl["n"])
        s = wl["solids"][0]
        o.add_sphere(s["center"], s["radius"], mu_w=mu_w, cavity=True)
        o.init_drops([c for c, _ in wl["drops"]], [r for _, r in wl["drops"]], W=10.0)
        o.step(2000)
        a = o.measure()
        assert a.status == 0 and a.n_valid == 2
        th.append(a.mean_deg)
    assert th[0] < 90.0 < th[2] and th[0] < th[1] < th[2], th


# ------------------------------- pseudopotential model (Sec. V: other models)

SC = dict(model=1, sc_G=W.SC_G, rho_l=W.SC_RHO_L, rho_g=W.SC_RHO_G)


def _sc_eos(rho, G):
    # the bulk pressure of the Shan-Chen interaction written with the lattice
    # weights: p = rho c_s^2 + G c_s^2 psi^2 / 2, c_s^2 = 1/3
    psi = 1.0 - math.exp(-rho)
    return rho / 3.0 + G * psi * psi / 6.0


@pytest.mark.parametrize("dim", [2, 3])
def test_sc_force_exact_on_quadratic_psi(dim):
    # the odd moments of the lattice weights vanish and the second ones are
    # c_s^2 I, so sum_i w_i psi(x + e_i) e_i = c_s^2 grad psi exactly when psi
    # is a quadratic: F = -G psi grad psi / 3 on every interior node
    o = O.Oracle(dim, (12, 11, 10 if dim == 3 else 1), **SC)
    zz, yy, xx = np.mgrid[0:o.shape[0], 0:o.shape[1], 0:o.shape[2]].astype(np.float64)
    psi = 0.3 + 0.01 * xx + 0.015 * yy + 0.002 * xx * xx - 0.001 * xx * yy + 0.0015 * yy * yy
    gx, gy, gz = 0.01 + 0.004 * xx - 0.001 * yy, 0.015 - 0.001 * xx + 0.003 * yy, 0.0 * xx
    if dim == 3:
        psi = psi + 0.01 * zz + 0.001 * zz * zz - 0.0007 * xx * zz
        gx, gz = gx - 0.0007 * zz, 0.01 + 0.002 * zz - 0.0007 * xx
    o.set_rho(-np.log(1.0 - psi))
    for ph in ("density", "fill", "mu", "force"):
        o.phase(ph)
    inner = (slice(1, -1) if dim == 3 else slice(None), slice(1, -1), slice(1, -1))
    F = o.force
    for ax, g in enumerate((gx, gy, gz)[:dim]):
        ref = -W.SC_G * psi * g / 3.0
        assert np.max(np.abs(F[ax][inner] - ref[inner])) < 1e-14, ax


def test_sc_flat_interface_has_equal_bulk_pressures():
    # a liquid slab relaxes until the momentum flux through the flat interface
    # balances: the bulk pressures of the two phases are equal (to 5e-13 after
    # 40,000 steps; 1e-6 after 20,000)
    o = O.Oracle(2, (128, 4), bgk=1, **SC)
    x = np.arange(128)
    r = 0.5 * (2.0 + 0.2) + 0.5 * (2.0 - 0.2) * np.tanh((32 - np.abs(x - 64.0)) / 2.0)
    o.set_rho(np.broadcast_to(r, (1, 4, 128)).copy())
    o.step(40000)
    o.update_derived()
    rl, rg = o.rho[0, 0, 64], o.rho[0, 0, 0]
    assert rl > 2.5 and rg < 0.1
    pl, pg = _sc_eos(rl, W.SC_G), _sc_eos(rg, W.SC_G)
    assert abs(pl - pg) < 1e-10 * pl, (rl, rg, pl, pg)
    assert abs(rl - W.SC_RHO_L) < 1e-3 and abs(rg - W.SC_RHO_G) < 1e-3


def test_sc_mass_and_wetting_order():
    # mass is conserved to round-off, and a denser wall wets more (Sec. V: the
    # measurement is the same for any model that yields a density field)
    th = []
    for rho_w in (0.4, 0.8, 1.3):
        wl = W.sc_sessile_2d(rho_w)
        o = O.Oracle(2, wl["n"], **SC)
        s = wl["solids"][0]
        o.add_sphere(s["center"], s["radius"], mu_w=rho_w)
        o.init_drops([c for c, _ in wl["drops"]], [r for _, r in wl["drops"]], W=wl["W"])
        m0 = o.mass()
        o.step(2500)
        assert abs(o.mass() / m0 - 1) < 1e-12
        a = o.measure()
        assert a.status == 0 and a.n_valid == 2
        th.append(a.mean_deg)
    assert th[0] > 120.0 and th[0] > th[1] > th[2] and th[2] < 70.0, th
