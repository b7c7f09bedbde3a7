"""Host-side reductions of the sweeps (no GPU): the relative L2 deviation from a
least-squares line (Sec. IV A) and the spherical-cap angle (Sec. IV A)."""
import math

import numpy as np

from paper_2202_06516_amd import sweeps as S


def test_linear_fit_error():
    x = np.linspace(-0.02, 0.16, 10)
    E, a, c = S.linear_fit_error(x, 470.0 * x + 75.0)
    assert E < 1e-14 and abs(a - 470.0) < 1e-9 and abs(c - 75.0) < 1e-9
    y = 470.0 * x + 75.0 + np.where(np.arange(10) % 2 == 0, 1.0, -1.0)
    E, a, c = S.linear_fit_error(x, y)
    F = a * x + c
    assert abs(E - np.linalg.norm(y - F) / np.linalg.norm(F)) < 1e-15 and 0.005 < E < 0.02


def test_cap_angle_of_a_circular_drop():
    # a tanh-profile circular drop meeting a circle at a known angle, with the
    # exact contact points: the cap construction recovers the angle
    ny, nx = 300, 400
    C, R = np.array([200.0, 60.0]), 80.0
    for theta in (60.0, 90.0, 120.0):
        # drop circle (centre on the axis, radius r) meeting the convex substrate at
        # theta: the angle between the two radii at an intersection is theta
        # (180 deg when the drop only touches the substrate from outside)
        r = 50.0
        g = math.radians(theta)
        D = math.sqrt(R * R + r * r - 2 * R * r * math.cos(g))
        c0 = C + np.array([0.0, D])
        yh = (R * R - r * r + D * D) / (2 * D)        # intersection height above C along the axis
        xh = math.sqrt(R * R - yh * yh)
        contact = [(C[0] + xh, C[1] + yh, 0.0), (C[0] - xh, C[1] + yh, 0.0)]
        yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
        rho = 0.5 - 0.5 * np.tanh((np.hypot(xx - c0[0], yy - c0[1]) - r) / 2.0)
        cls = np.where(np.hypot(xx - C[0], yy - C[1]) <= R, 1, 0).astype(np.uint8)
        cap = S.cap_angle(rho, cls, 0.5, C, R, contact)
        assert abs(cap - theta) < 0.5, (theta, cap)


def test_sliding_drop_starts_tangent_to_the_plate():
    # the drop of the sliding-drop run touches the arc from above at x0: its
    # centre lies on the arc's normal, r0 beyond it
    from paper_2202_06516_amd import rolling as RL
    cx, cy, R, r0 = 1500.0, 1.5 + 100.0 - 6000.0, 6000.0, 100.0
    for x0 in (600.0, 900.0, 1500.0, 2100.0):
        px, py = RL.start_drop(cx, cy, R, x0, r0)
        assert abs(math.hypot(px - cx, py - cy) - (R + r0)) < 1e-9
        ys = cy + math.sqrt(R * R - (x0 - cx) ** 2)
        assert abs(math.hypot(px - x0, py - ys) - r0) < 1e-9


def test_bump_geometry():
    # a bump of radius R rising H above the floor at y = 1.5 has the width
    # L = 2 sqrt(2 R H - H^2) there, and the drop sits tangent on its top
    from paper_2202_06516_amd import workloads as W
    cs = W.bump_case(700, 400, 150.0, 100.0, 40.0, 0.04)
    (cx, cy), R = cs["solid"]["center"], cs["solid"]["radius"]
    assert abs(cy + R - (1.5 + 100.0)) < 1e-12
    half = math.sqrt(R * R - (1.5 - cy) ** 2)
    assert abs(2 * half - 2 * math.sqrt(2 * 150.0 * 100.0 - 100.0 ** 2)) < 1e-9
    (dx, dy), r0 = cs["drop"]
    assert dx == cx and abs(dy - r0 - (cy + R)) < 1e-12
