"""Batched solver: every case equals the same case run alone, bit for bit."""
import math

import numpy as np
import pytest

from paper_2202_06516_amd import lbm as G
from paper_2202_06516_amd import workloads as W

from .pairs import BASE, gpu_lattice, oracle_lattice, rel_err

pytestmark = pytest.mark.gpu

PHYS = dict(BASE, Tr=0.8)


def small_cases(n=5, seed=7):
    cases, _ = W.batch_cases(n, seed=seed, nmin=64, nmax=112, rs=(8.0, 14.0), r0=(7.0, 11.0), mu=(-0.01, 0.1))
    return cases


def single(case, precision, **kw):
    wl = dict(dim=2, n=case["n"], wall=(0, 0), solids=[case["solid"]], drops=[case["drop"]])
    return gpu_lattice(wl, precision, **kw)


@pytest.mark.parametrize("precision", [G.LBM_F64, G.LBM_F32])
def test_batch_equals_single(precision):
    cases = small_cases()
    b = G.Batch(cases, precision=precision, tile_w=128, blocks_per_cu=2, **PHYS)
    b.step(45, measure_every=15)
    b.sync()
    ang = b.angles()
    for i, cs in enumerate(cases):
        s = single(cs, precision, Tr=0.8)
        sa = s.step(45, measure_every=15, cap=4)
        fb, fs = b.read(i, G.FIELD_F), s.f
        assert np.array_equal(fb, fs), f"case {i}: max diff {np.abs(fb - fs).max()}"
        assert np.array_equal(b.read(i, G.FIELD_RHO), s.rho)
        last = sa[-1]
        assert ang[i].step == last.step == 30
        for k in range(2):
            x, y = ang[i].sector_deg[k], last.sector_deg[k]
            assert (math.isnan(x) and math.isnan(y)) or x == y


def test_batch_case_against_oracle():
    cases = small_cases(3, seed=11)
    b = G.Batch(cases, precision=G.LBM_F64, **PHYS)
    b.step(20)
    for i, cs in enumerate(cases):
        wl = dict(dim=2, n=cs["n"], wall=(0, 0), solids=[cs["solid"]], drops=[cs["drop"]])
        o = oracle_lattice(wl, Tr=0.8)
        o.step(20)
        o.update_derived()
        assert rel_err(b.read(i, G.FIELD_RHO), o.rho, o.cls == 0) < 1e-12


def test_launch_shape_does_not_change_results(tmp_path):
    cases = small_cases(4, seed=3)
    a = G.Batch(cases, precision=G.LBM_F32, tile_w=64, blocks_per_cu=4, **PHYS)
    c = G.Batch(cases, precision=G.LBM_F32, autotune=True, cache_path=str(tmp_path / "tune.json"), **PHYS)
    inf = c.info()
    assert inf["tile_w"] in (64, 128, 256) and 1 <= inf["blocks_per_cu"] <= 32
    a.step(40)
    c.step(40)
    for i in range(len(cases)):
        assert np.array_equal(a.read(i, G.FIELD_F), c.read(i, G.FIELD_F))
    # the cached choice is reused
    d = G.Batch(cases, precision=G.LBM_F32, autotune=True, cache_path=str(tmp_path / "tune.json"), **PHYS)
    assert (d.info()["tile_w"], d.info()["blocks_per_cu"]) == (inf["tile_w"], inf["blocks_per_cu"])


def test_batch_warm_write():
    cases = small_cases(3, seed=5)
    b = G.Batch(cases, precision=G.LBM_F64, **PHYS)
    b.step(10)
    rho = b.read(1, G.FIELD_RHO)
    b.write_rho(1, rho)
    s = single(cases[1], G.LBM_F64, Tr=0.8)
    s.step(10)
    s.write(G.FIELD_RHO, s.rho)
    b.step(7)
    s.step(7)
    assert np.array_equal(b.read(1, G.FIELD_F), s.f)


@pytest.mark.parametrize("precision", [G.LBM_F32, G.LBM_F64])
def test_device_writes_equal_host_writes(precision):
    # Densities handed over as device pointers from one staging buffer that the
    # caller refills right after each call: every copy must be complete and
    # ordered with the library's own kernels when the call returns.
    torch = pytest.importorskip("torch")
    cases = small_cases(6, seed=11)
    dt = np.float64 if precision == G.LBM_F64 else np.float32
    fields = []
    for i, c in enumerate(cases):
        nx, ny = c["n"]
        x = np.arange(nx)[None, :]
        y = np.arange(ny)[:, None]
        cx, cy = c["drop"][0]
        r = np.hypot(x - cx, y - cy)
        fields.append((0.5 * (0.2 + 7.0) - 3.4 * np.tanh((r - c["drop"][1] - 0.3 * i) / 3.0)).astype(dt))
    host = G.Batch(cases, precision=precision, **PHYS)
    dev = G.Batch(cases, precision=precision, **PHYS)
    cap = max(f.size for f in fields)
    stage = torch.empty(cap, dtype=torch.float64 if dt == np.float64 else torch.float32, device="cuda")
    for i, f in enumerate(fields):
        host.write_rho(i, f)
        n = f.size
        stage[:n].copy_(torch.from_numpy(f.reshape(-1)))
        torch.cuda.synchronize()
        dev.write_rho_device(i, stage.data_ptr(), n * f.itemsize)
        stage.fill_(float("nan"))          # the caller reuses its buffer at once
        torch.cuda.synchronize()
    for b in (host, dev):
        b.step(25)
        b.sync()
    for i in range(len(cases)):
        assert np.array_equal(host.read(i, G.FIELD_F), dev.read(i, G.FIELD_F)), i
    # the single-lattice entry point: the same contract
    s_host = single(cases[2], precision, Tr=0.8)
    s_dev = single(cases[2], precision, Tr=0.8)
    s_host.write(G.FIELD_RHO, fields[2])
    stage[:fields[2].size].copy_(torch.from_numpy(fields[2].reshape(-1)))
    torch.cuda.synchronize()
    s_dev.write_device(G.FIELD_RHO, stage.data_ptr(), fields[2].nbytes)
    stage.fill_(float("nan"))
    torch.cuda.synchronize()
    s_host.step(25)
    s_dev.step(25)
    assert np.array_equal(s_host.f, s_dev.f)


def test_profiled_steps_are_ordinary_steps():
    # lbm_batch_profile_step times the three main kernels over eager steps; the
    # state it leaves equals that of the same number of ordinary steps
    cases = small_cases(3, seed=13)
    a = G.Batch(cases, precision=G.LBM_F32, **PHYS)
    c = G.Batch(cases, precision=G.LBM_F32, **PHYS)
    prof = a.profile(7)
    assert set(prof) == {"kb_density", "kb_mu", "kb_collide"}
    assert all(v > 0.0 for v in prof.values())
    c.step(7)
    c.sync()
    assert a.info()["step"] == c.info()["step"] == 7
    for i in range(len(cases)):
        assert np.array_equal(a.read(i, G.FIELD_F), c.read(i, G.FIELD_F))


@pytest.mark.parametrize("precision", [G.LBM_F64, G.LBM_F32])
def test_batch_d3q19_equals_single(precision):
    # three-dimensional cases (spheres, one cavity) in one batch: populations
    # bit for bit and the 16-sector angles of the lone lattices
    cases = [
        dict(n=(40, 36, 40), solid=dict(center=(20.2, 18.1, 10.3), radius=7.4, mu_w=0.04),
             drop=((20.0, 18.0, 25.0), 7.0)),
        dict(n=(48, 40, 44), solid=dict(center=(24.0, 20.0, 22.0), radius=19.0, mu_w=0.02, cavity=True),
             drop=((24.0, 20.0, 11.0), 8.0)),
        dict(n=(36, 36, 36), solid=dict(center=(18.0, 18.0, 9.5), radius=6.0, mu_w=-0.01),
             drop=((18.0, 18.0, 21.0), 7.5)),
    ]
    params = dict(PHYS, collision=G.LBM_BGK)
    b = G.Batch(cases, lattice=G.LBM_D3Q19, precision=precision, **params)
    b.step(30, measure_every=15)
    b.sync()
    ang = b.angles()
    for i, cs in enumerate(cases):
        wl = dict(dim=3, n=cs["n"], wall=(0, 0, 0), solids=[cs["solid"]], drops=[cs["drop"]])
        s = gpu_lattice(wl, precision, "bgk", Tr=0.8)
        s.set_measure(0, 16)
        sa = s.step(30, measure_every=15, cap=4)
        assert np.array_equal(b.read(i, G.FIELD_F), s.f), i
        assert np.array_equal(b.read(i, G.FIELD_CLASS), s.read(G.FIELD_CLASS))
        last = sa[-1]
        assert ang[i].step == last.step and ang[i].status == last.status
        for k in range(16):
            x, y = ang[i].sector_deg[k], last.sector_deg[k]
            assert (math.isnan(x) and math.isnan(y)) or abs(x - y) <= 1e-9, (i, k, x, y)
