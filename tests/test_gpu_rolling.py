"""A drop sliding on a tilted curved plate (Sec. IV D), reduced to a 600 x 160 box."""
import math

import pytest

from paper_2202_06516_amd import rolling as RL

pytestmark = pytest.mark.gpu


def test_drop_slides_downhill_with_advancing_side_downhill():
    # r0 = 30 on an arc of R = 1200 rising 40 lu, gravity tilted by 20 deg
    # toward +x: after the gravity-free relaxation the drop moves along +x,
    # the library's advancing side is the downhill contact line at every
    # sample, and the angles stay near the plate's intrinsic angle
    rep = RL.run(nx=600, ny=160, R=1200.0, H=40.0, r0=30.0, x0=200.0, mu_w=0.063, g=4e-6, phi_deg=20.0, Tr=0.8,
                 relax=5000, steps=60000, every=500, chunk=5000, log=lambda s: None)
    print({k: v for k, v in rep.items() if k != "records"})
    ok = [r for r in rep["records"] if r["status"] == 0]
    assert len(ok) >= 0.9 * len(rep["records"])
    assert rep["library_sides"]
    assert rep["travel"] > 20.0
    assert 100.0 < rep["theta_a_mean"] < 145.0 and 100.0 < rep["theta_r_mean"] < 145.0
    assert all(math.isfinite(r["theta_a"]) and math.isfinite(r["theta_r"]) for r in ok)
