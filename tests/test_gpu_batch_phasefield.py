"""The phase-field model in the batched solver: every case equals the same case
advanced alone (whose model the oracle pins, test_gpu_phasefield.py), bit for
bit: both population sets, phi, rho and the in-step angles read on phi."""
import math

import numpy as np
import pytest

from paper_2202_06516_amd import lbm as G
from paper_2202_06516_amd import workloads as W

from .pairs import BASE, gpu_lattice, oracle_lattice, rel_err

pytestmark = pytest.mark.gpu

PF = dict(BASE, model=G.LBM_MODEL_PHASE_FIELD, **W.PF_PARAMS)


def pf_cases(n=4, seed=21):
    # the layout of the chemical-potential cases; the wall value of each solid
    # is a wall order parameter, seeded in [-0.4, 0.4]
    cases, _ = W.batch_cases(n, seed=seed, nmin=64, nmax=112, rs=(8.0, 14.0), r0=(7.0, 11.0))
    return W.pf_batch_cases(cases, seed + 1)


def single(case, precision, dim=2, collision="mrt", bc="halfway"):
    wl = dict(dim=dim, n=case["n"], wall=(0,) * dim, model=2, W=W.PF_W, solids=[case["solid"]],
              drops=[case["drop"]])
    return gpu_lattice(wl, precision, collision, bc)


def same_angles(a, b):
    for k in range(a.n_sectors):
        x, y = a.sector_deg[k], b.sector_deg[k]
        assert (math.isnan(x) and math.isnan(y)) or x == y, (k, x, y)


@pytest.mark.parametrize("precision", [G.LBM_F64, G.LBM_F32])
def test_pf_batch_equals_single(precision):
    cases = pf_cases()
    b = G.Batch(cases, precision=precision, tile_w=128, blocks_per_cu=2, **PF)
    b.step(60, measure_every=20)
    b.sync()
    ang = b.angles()
    for i, cs in enumerate(cases):
        s = single(cs, precision)
        s.set_measure(0, 2)
        sa = s.step(60, measure_every=20, cap=4)
        for field, ref in ((G.FIELD_F, s.f), (G.FIELD_G, s.g), (G.FIELD_PHI, s.phi), (G.FIELD_RHO, s.rho)):
            got = b.read(i, field)
            assert np.array_equal(got, ref), (i, field, float(np.abs(got - ref).max()))
        assert ang[i].step == sa[-1].step == 40
        same_angles(ang[i], sa[-1])
    assert any(a.n_valid == 2 for a in ang)


def test_pf_batch_case_against_oracle():
    cases = pf_cases(2, seed=5)
    b = G.Batch(cases, precision=G.LBM_F64, **PF)
    b.step(30)
    for i, cs in enumerate(cases):
        wl = dict(dim=2, n=cs["n"], wall=(0, 0), model=2, W=W.PF_W, solids=[cs["solid"]], drops=[cs["drop"]])
        o = oracle_lattice(wl)
        o.step(30)
        o.update_derived()
        assert rel_err(b.read(i, G.FIELD_PHI), o.phi, o.cls <= 2) < 1e-12
        assert rel_err(b.read(i, G.FIELD_G), o.g) < 1e-12


def test_pf_batch_d3q19_equals_single():
    cases = [
        dict(n=(40, 36, 40), solid=dict(center=(20.2, 18.1, 10.3), radius=7.4, mu_w=0.3),
             drop=((20.0, 18.0, 25.0), 7.0)),
        dict(n=(36, 40, 36), solid=dict(center=(18.0, 20.0, 9.5), radius=6.0, mu_w=-0.2),
             drop=((18.0, 20.0, 21.0), 7.5)),
    ]
    b = G.Batch(cases, lattice=G.LBM_D3Q19, precision=G.LBM_F32, collision=G.LBM_BGK, **PF)
    b.step(40, measure_every=20)
    b.sync()
    ang = b.angles()
    for i, cs in enumerate(cases):
        s = single(cs, G.LBM_F32, dim=3, collision="bgk")
        s.set_measure(0, 16)
        sa = s.step(40, measure_every=20, cap=3)
        assert np.array_equal(b.read(i, G.FIELD_F), s.f), i
        assert np.array_equal(b.read(i, G.FIELD_G), s.g), i
        same_angles(ang[i], sa[-1])


def test_pf_batch_write_phi_and_profile():
    cases = pf_cases(3, seed=9)
    b = G.Batch(cases, precision=G.LBM_F64, **PF)
    b.step(11)
    phi = b.read(1, G.FIELD_PHI)
    b.write_phi(1, phi)
    s = single(cases[1], G.LBM_F64)
    s.step(11)
    s.write(G.FIELD_PHI, s.phi)
    # the other cases keep their state: against their lone lattices after 11 + 7 steps
    prof = b.profile(7)
    assert set(prof) == {"kb_pf_density", "kb_pf_mu", "kb_pf_collide"}
    s.step(7)
    assert np.array_equal(b.read(1, G.FIELD_F), s.f) and np.array_equal(b.read(1, G.FIELD_G), s.g)
    other = single(cases[2], G.LBM_F64)
    other.step(18)
    assert np.array_equal(b.read(2, G.FIELD_G), other.g)
    with pytest.raises(G.LbmError):
        b.write_rho(0, phi)
    with pytest.raises(G.LbmError):
        G.Batch(cases, precision=G.LBM_F64, **dict(PF, pf_tau=0.5))


def test_pf_batch_interpolated_wall_and_in_step_young():
    # the fluid populations on the interpolated wall (the order parameter
    # halfway), and the Young force at every in-step measurement read on phi
    # (band -0.8..0.8): each case against its lone lattice, bit for bit
    cases = pf_cases(3, seed=31)
    cases[1]["solid"] = dict(cases[1]["solid"], stripes=(-0.3, 0.25, 7.0))
    cases[1]["solid"].pop("mu_w")
    b = G.Batch(cases, precision=G.LBM_F64, bc_mode=G.LBM_BC_BOUZIDI_MC, **PF)
    b.set_young(0.0133, 70.0, 110.0)
    b.step(90, measure_every=30)
    by, ang = b.young_last(), b.angles()
    da, dy = b.young_force(0.0133, 70.0, 110.0)   # on demand, at step 90
    for i, cs in enumerate(cases):
        s = single(cs, G.LBM_F64, bc="bouzidi")
        s.set_measure(0, 2)
        s.set_young(0.0133, 70.0, 110.0)
        sa = s.step(90, measure_every=30, cap=4)
        sy = s.young_series()[-1]
        assert np.array_equal(b.read(i, G.FIELD_F), s.f), i
        assert np.array_equal(b.read(i, G.FIELD_G), s.g), i
        same_angles(ang[i], sa[-1])
        assert by[i].step == sy.step == 60 and by[i].status == sy.status
        for k in range(2):
            assert list(by[i].count[k]) == list(sy.count[k]), (i, k)
            for name in ("phi_d", "theta_eq_deg", "force"):
                g, r = getattr(by[i], name)[k], getattr(sy, name)[k]
                assert (math.isnan(g) and math.isnan(r)) or g == r, (i, k, name, g, r)
        oa, oy = s.young_force(0.0133, 70.0, 110.0)
        same_angles(da[i], oa)
        assert dy[i].status == oy.status
        for k in range(2):
            assert list(dy[i].count[k]) == list(oy.count[k]), (i, k)
            g, r = dy[i].force[k], oy.force[k]
            assert (math.isnan(g) and math.isnan(r)) or g == r, (i, k, g, r)
    assert any(sum(y.count[0]) + sum(y.count[1]) > 0 for y in by)
