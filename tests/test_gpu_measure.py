"""GPU contact-angle measurement against the oracle and against exact geometry."""
import math

import numpy as np
import pytest

from paper_2202_06516_amd import lbm as G
from paper_2202_06516_amd import workloads as W

from .pairs import BASE, gpu_lattice, oracle_lattice, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [G.LBM_F64, G.LBM_F32])
@pytest.mark.parametrize("theta0", [30, 60, 90, 120, 150])
def test_wedge_exact(precision, theta0):
    wl = dict(dim=2, n=(200, 180), wall=(0, 0), solids=[dict(center=(100, 60), radius=60, mu_w=0.0)], drops=[])
    gp = gpu_lattice(wl, precision)
    inf = gp.info()
    rho = W.wedge_density(gp.shape, (100, 60), 60, theta0, inf["rho_m"], inf["rho_g"], inf["rho_l"])
    gp.write(G.FIELD_RHO, rho)
    a = gp.measure()
    assert a.status == 0 and a.n_valid == 2
    tol = 1e-9 if precision == G.LBM_F64 else 2e-3
    assert abs(a.sector_deg[0] - theta0) < tol
    assert abs(a.sector_deg[1] - theta0) < tol
    o = oracle_lattice(wl)
    o.set_rho(rho)
    b = o.measure()
    assert abs(a.sector_deg[0] - b.sector_deg[0]) < tol


def test_no_contact_line():
    wl = dict(dim=2, n=(64, 64), wall=(0, 0), solids=[dict(center=(32, 16), radius=8, mu_w=0.0)], drops=[])
    gp = gpu_lattice(wl, G.LBM_F64)
    gp.write(G.FIELD_RHO, np.full(gp.shape, gp.info()["rho_g"]))
    a = gp.measure()
    assert a.status == G.LBM_E_NO_CONTACT_LINE and math.isnan(a.mean_deg)


def test_sessile_2d_full_run():
    """The 128^2 FP64 workload, 5000 steps, angle every 100 steps (Tr = 0.6)."""
    wl = W.sessile_2d(mu_w=0.04)
    gp = gpu_lattice(wl, G.LBM_F64)
    o = oracle_lattice(wl)
    ga = gp.step(wl["steps"], measure_every=wl["every"], cap=64)
    oa = o.step_measured(wl["steps"], wl["every"], 0, 2)
    assert len(ga) == len(oa) == 50
    worst = 0.0
    for a, b in zip(ga, oa):
        assert a.step == b.step and a.status == b.status
        for s in range(2):
            x, y = a.sector_deg[s], b.sector_deg[s]
            if math.isnan(y):
                assert math.isnan(x)
                continue
            worst = max(worst, abs(x - y))
    assert worst < 1e-6, worst
    o.update_derived()
    assert rel_err(gp.rho, o.rho, (o.cls == 0) | (o.cls == 1) | (o.cls == 2)) < 1e-10
    last = ga[-1]
    # mirror symmetry of the layout: both sides agree
    assert abs(last.sector_deg[0] - last.sector_deg[1]) < 1e-6
    assert 90.0 < last.mean_deg < 110.0


@pytest.mark.parametrize("precision,tol", [(G.LBM_F64, 1e-6), (G.LBM_F32, 0.1)])
def test_sessile_3d_small_sectors(precision, tol):
    wl = W.sessile_3d(mu_w=0.04, n=80)
    gp = gpu_lattice(wl, precision, "bgk", Tr=0.8)
    gp.set_measure(0, 8)
    o = oracle_lattice(wl, "bgk", Tr=0.8)
    ga = gp.step(120, measure_every=40, cap=8)
    oa = o.step_measured(120, 40, 0, 8)
    assert len(ga) == len(oa) == 3
    for a, b in zip(ga[1:], oa[1:]):
        assert a.n_valid == b.n_valid and a.n_valid >= 6
        ds = [abs(a.sector_deg[s] - b.sector_deg[s]) for s in range(8) if not math.isnan(b.sector_deg[s])]
        assert max(ds) < tol, ds
        assert abs(a.mean_deg - b.mean_deg) < tol


def test_gravity_advancing_receding():
    wl = W.sessile_2d(mu_w=0.04)
    g = (1e-6, 0.0, 0.0)
    gp = gpu_lattice(wl, G.LBM_F64, g=g, g_start=0)
    o = oracle_lattice(wl, g=g, g_start=0)
    gp.step(400)
    o.step(400)
    a = gp.measure()
    b = o.measure()
    assert abs(a.adv_deg - b.adv_deg) < 1e-6 and abs(a.rec_deg - b.rec_deg) < 1e-6
    # g points to +x: the advancing side is the right-hand one (sector 0)
    assert a.adv_deg == a.sector_deg[0]


# ------------------------------------------- unbalanced Young force (Eq. 17, 18)


def _young_pair(gy, oy, ga, oa, tol):
    assert gy.status == oy.status == 0
    for s in range(ga.n_sectors):
        assert list(gy.count[s]) == list(oy.count[s]), (s, list(gy.count[s]), list(oy.count[s]))
        for name in ("phi_d", "theta_eq_deg", "force"):
            g, o = getattr(gy, name)[s], getattr(oy, name)[s]
            assert (math.isnan(g) and math.isnan(o)) or abs(g - o) <= tol, (name, s, g, o)


@pytest.mark.parametrize("width", [20.0, 60 * math.pi / 6, 100.0])
def test_young_force_on_wedge_matches_oracle(width):
    # the exact wedge on a striped circle: the footprint entirely on the
    # second stripe, split by a border, entirely on the first stripe
    sol = dict(center=(100, 60), radius=60, stripes=(0.0, 0.05, width))
    wl = dict(dim=2, n=(200, 180), wall=(0, 0), solids=[sol], drops=[])
    gp = gpu_lattice(wl, G.LBM_F64)
    gp.set_measure(0, 2)
    inf = gp.info()
    rho = W.wedge_density(gp.shape, (100, 60), 60, 90, inf["rho_m"], inf["rho_g"], inf["rho_l"], slope=1.0)
    gp.write(G.FIELD_RHO, rho)
    ga, gy = gp.young_force(0.05, 70.0, 130.0)
    o = oracle_lattice(wl)
    o.set_rho(rho)
    oa, oy = o.young_force(0.05, 70.0, 130.0)
    _young_pair(gy, oy, ga, oa, 1e-12)
    assert sum(gy.count[0]) > 0


def test_young_force_on_relaxing_striped_drops():
    # a drop relaxing on a striped cylinder (2-D, two sides) and a striped
    # sphere (3-D, 8 sectors): footprint counts bit-exact, phi_d / theta_eq /
    # force to round-off (FP64)
    wl2 = dict(dim=2, n=(96, 80), wall=(0, 0), Tr=0.8,
               solids=[dict(center=(48.3, 24.6), radius=16.2, stripes=(-0.01, 0.08, 9.0))],
               drops=[((48.0, 52.0), 12.0)])
    wl3 = dict(dim=3, n=(48, 44, 46), wall=(1, 1, 1), Tr=0.8,
               solids=[dict(center=(24.2, 22.1, 15.3), radius=9.1, stripes=(-0.01, 0.08, 5.0))],
               drops=[((24.0, 22.0, 30.0), 8.0)])
    for wl, ns, coll in ((wl2, 2, "mrt"), (wl3, 8, "bgk")):
        gp = gpu_lattice(wl, G.LBM_F64, coll)
        gp.set_measure(0, ns)
        o = oracle_lattice(wl, coll)
        gp.step(150)
        o.step(150)
        ga, gy = gp.young_force(0.06, 80.0, 120.0, roughness=1.0)
        oa, oy = o.young_force(0.06, 80.0, 120.0, n_sectors=ns)
        assert ga.n_valid == oa.n_valid and ga.n_valid >= 1
        _young_pair(gy, oy, ga, oa, 1e-9)


def test_young_force_without_contact_line_and_bad_options():
    wl = dict(dim=2, n=(64, 64), wall=(0, 0), solids=[dict(center=(32, 16), radius=8, mu_w=0.0)], drops=[])
    gp = gpu_lattice(wl, G.LBM_F64)
    gp.write(G.FIELD_RHO, np.full(gp.shape, gp.info()["rho_g"]))
    a, y = gp.young_force(0.05, 90.0)
    assert y.status == G.LBM_E_NO_CONTACT_LINE and math.isnan(y.phi_d[0]) and math.isnan(y.force[1])
    for kw in (dict(roughness=0.0), dict(band=(0.5, 0.4)), dict(band=(0.0, 1.0))):
        with pytest.raises(G.LbmError):
            gp.young_force(0.05, 90.0, **kw)


def test_batch_young_force_equals_single_lattices():
    # every case of a batch (uniform cylinder, striped cylinder, cavity) gives
    # the footprint counts, phi_d, theta_eq and forces of the same case run alone
    cases = [
        dict(n=(96, 80), solid=dict(center=(48.3, 24.6), radius=16.2, mu_w=0.04), drop=((48.0, 52.0), 12.0)),
        dict(n=(96, 80), solid=dict(center=(48.3, 24.6), radius=16.2, stripes=(-0.01, 0.08, 9.0)),
             drop=((48.0, 52.0), 12.0)),
        dict(n=(70, 52), solid=dict(center=(35.3, 26.1), radius=23.4, mu_w=0.04, cavity=True), drop=((35.0, 12.0), 9.0)),
    ]
    b = G.Batch(cases, precision=G.LBM_F64, **dict(BASE, Tr=0.8))
    b.step(150)
    ba, by = b.young_force(0.06, 80.0, 120.0)
    for i, cs in enumerate(cases):
        wl = dict(dim=2, n=cs["n"], wall=(0, 0), solids=[cs["solid"]], drops=[cs["drop"]])
        s = gpu_lattice(wl, G.LBM_F64, Tr=0.8)
        s.set_measure(0, 2)
        s.step(150)
        sa, sy = s.young_force(0.06, 80.0, 120.0)
        assert by[i].status == sy.status == 0 and ba[i].step == sa.step
        for k in range(2):
            assert list(by[i].count[k]) == list(sy.count[k]), (i, k)
            for name in ("phi_d", "theta_eq_deg", "force"):
                g, r = getattr(by[i], name)[k], getattr(sy, name)[k]
                assert (math.isnan(g) and math.isnan(r)) or abs(g - r) <= 1e-12, (i, k, name, g, r)
    assert sum(by[1].count[0]) > 0 and by[0].phi_d[0] == 1.0
    with pytest.raises(G.LbmError):
        b.young_force(0.06, 80.0, 120.0, roughness=0.0)


def test_young_force_in_step_matches_oracle():
    # the Young force taken at every in-step measurement (every 100 steps of a
    # drop relaxing on a striped cylinder) equals the oracle's Eq. 17-18 on the
    # same states: counts bit-exact, phi_d / theta_eq / force to round-off
    wl = dict(dim=2, n=(96, 80), wall=(0, 0), Tr=0.8,
              solids=[dict(center=(48.3, 24.6), radius=16.2, stripes=(-0.01, 0.08, 9.0))],
              drops=[((48.0, 52.0), 12.0)])
    gp = gpu_lattice(wl, G.LBM_F64)
    gp.set_measure(0, 2)
    gp.set_young(0.06, 80.0, 120.0)
    ga = gp.step(1000, measure_every=100, cap=16)
    gy = gp.young_series()
    assert len(ga) == len(gy) == 10
    o = oracle_lattice(wl)
    for k in range(10):
        oa, oy = o.young_force(0.06, 80.0, 120.0)
        assert gy[k].step == ga[k].step == oy.step == 100 * k and gy[k].status == oy.status
        for s in range(2):
            assert list(gy[k].count[s]) == list(oy.count[s]), (k, s)
            for name in ("phi_d", "theta_eq_deg", "force"):
                g, r = getattr(gy[k], name)[s], getattr(oy, name)[s]
                assert (math.isnan(g) and math.isnan(r)) or abs(g - r) <= 1e-9, (k, s, name, g, r)
        o.step(100)
    assert any(sum(gy[k].count[0]) > 0 for k in range(10))
    gp.set_young(None)
    with pytest.raises(G.LbmError):
        gp.young_series()
    for kw in (dict(roughness=0.0), dict(band=(0.5, 0.4)), dict(band=(0.0, 1.0))):
        with pytest.raises(G.LbmError):
            gp.set_young(0.06, 80.0, 120.0, **kw)


def test_batch_in_step_young_force_equals_single():
    # the in-step Young force of every case of a batch equals that of the same
    # case run alone (latest record after three measurements)
    cases = [
        dict(n=(96, 80), solid=dict(center=(48.3, 24.6), radius=16.2, stripes=(-0.01, 0.08, 9.0)),
             drop=((48.0, 52.0), 12.0)),
        dict(n=(70, 52), solid=dict(center=(35.3, 26.1), radius=23.4, mu_w=0.04, cavity=True), drop=((35.0, 12.0), 9.0)),
    ]
    b = G.Batch(cases, precision=G.LBM_F64, **dict(BASE, Tr=0.8))
    b.set_young(0.06, 80.0, 120.0)
    assert all(y.status == G.LBM_E_NO_CONTACT_LINE for y in b.young_last())
    b.step(300, measure_every=100)
    by = b.young_last()
    for i, cs in enumerate(cases):
        wl = dict(dim=2, n=cs["n"], wall=(0, 0), solids=[cs["solid"]], drops=[cs["drop"]])
        s = gpu_lattice(wl, G.LBM_F64, Tr=0.8)
        s.set_measure(0, 2)
        s.set_young(0.06, 80.0, 120.0)
        s.step(300, measure_every=100, cap=4)
        sy = s.young_series()[-1]
        assert by[i].step == sy.step == 200 and by[i].status == sy.status == 0
        for k in range(2):
            assert list(by[i].count[k]) == list(sy.count[k]), (i, k)
            for name in ("phi_d", "theta_eq_deg", "force"):
                g, r = getattr(by[i], name)[k], getattr(sy, name)[k]
                assert (math.isnan(g) and math.isnan(r)) or abs(g - r) <= 1e-12, (i, k, name, g, r)
    b.set_young(None)
    with pytest.raises(G.LbmError):
        b.young_last()


@pytest.mark.parametrize("n", [(48, 44, 46), (64, 44, 46)])
@pytest.mark.parametrize("precision", [G.LBM_F32, G.LBM_F32_MIXED])
def test_young_force_in_step_3d_fp32_matches_oracle(n, precision):
    # the in-step Young force on a striped sphere in 3-D (8 sectors; the
    # split step at nx = 48, the one-pass step at nx = 64) with FP32 storage:
    # each record equals the oracle's Eq. 17-18 on the density the GPU held at
    # that step (counts bit-exact, phi_d / theta_eq / force to round-off)
    c = (n[0] / 2 + 0.3, 22.2, 17.4)
    wl = dict(dim=3, n=n, wall=(1, 1, 1), Tr=0.8, solids=[dict(center=c, radius=11.0, stripes=(-0.01, 0.08, 3.0))],
              drops=[((c[0] - 0.2, c[1] - 0.1, c[2] + 11.0 + 8.0 - 1.6), 8.0)])
    gp = gpu_lattice(wl, precision, "bgk")
    gp.set_measure(0, 8)
    gp.set_young(0.06, 80.0, 120.0)
    o = oracle_lattice(wl, "bgk")
    every, checked = 40, 0
    for k in range(6):
        rho = gp.rho  # the state the next call measures at its first step
        ga = gp.step(every, measure_every=every, cap=2)
        gy = gp.young_series()
        assert len(ga) == len(gy) == 1 and gy[0].step == ga[0].step == every * k
        o.set_rho(rho)
        oa, oy = o.young_force(0.06, 80.0, 120.0, n_sectors=8)
        assert gy[0].status == oy.status
        for s in range(8):
            assert list(gy[0].count[s]) == list(oy.count[s]), (k, s)
            for name in ("phi_d", "theta_eq_deg", "force"):
                g, r = getattr(gy[0], name)[s], getattr(oy, name)[s]
                assert (math.isnan(g) and math.isnan(r)) or abs(g - r) <= 1e-9, (k, s, name, g, r)
        checked += sum(1 for s in range(8) if not math.isnan(oy.force[s]))
    assert checked > 0
