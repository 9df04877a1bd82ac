"""Wetting by virtual wall density on the GPU path (Sec. 4.5).

- The Young-Laplace column of the oracle pin, run through the library: FP64 parity with
  the oracle, and the library's calibration module measuring the same angles as the
  test-side analysis of the oracle's field.
- The calibration in the wettability-driven column's channel (H = 70, nu = 0.075): the
  meniscus angle and the angle from the pressure jump agree, and the inverse map returns
  wall densities that give the requested angles.
- The wettability-driven column (H = 70, L = 1260, L_l = 420, nu_l = nu_v = 0.075, angles
  59.3 -> 63.4 degrees on the right half): centroid motion against the closed form of
  Esmaili et al. the paper compares with. The density ratio is 16.7 (van der Waals at
  T/Tc = 0.7), not the paper's 10^3: with virtual-density walls this model diverges for
  wall densities far from the adjacent phase beyond a ratio of about 25 (measured map in
  the design notes).
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import lbm_inputs as L
from oracle import oracle as O
from oracle import thermo as T
from tests import wetting_analysis as WA
from tests.gpu_cases import max_rel

pytestmark = pytest.mark.gpu

A9, B21 = 9 / 49, 2 / 21


def _fluid(P, tr, W, tau):
    base = P.Params(P.LBM_D2Q9, 8, 4, 1, P.LBM_EOS_VDW, A9, B21, 1.0, 0.0, tr, 0.02, tau)
    a = A9 * 0.02 / P.lbm_kappa_for_width(base, W)
    return P.Params(P.LBM_D2Q9, 8, 4, 1, P.LBM_EOS_VDW, a, B21, 1.0, 0.0, tr, 0.02, tau)


def test_young_laplace_column_parity_and_angles():
    import paper_2112_01975_amd as P
    from paper_2112_01975_amd import wetting as Wt
    tr, W, H, nw, nx, steps = 0.7, 4.0, 24, 2, 72, 8000
    base = _fluid(P, tr, W, 0.8)
    fl = T.Fluid(T.VDW, base.a, B21, tr)
    rv, rl, _ = T.coexistence(fl)
    mask, rho0 = L.channel_column(nx, H, nw, rl, rv, W, nx / 3, 2 * nx / 3)
    ny = H + 2 * nw
    rw = rv + 0.3 * (rl - rv)
    cfg = O.Config(2, nx, ny, 1, T.VDW, base.a, B21, 1.0, 0.0, tr, 0.02, 0.8, rho_wall=rw)
    r_o, U_o, _ = O.Oracle(cfg, mask).init(rho0).step(steps).moments()
    p = replace(base, nx=nx, ny=ny, mask=mask, rho_wall=rw)
    with P.Simulation(p) as s:
        s.init(rho0)
        s.step(steps)
        r_g, U_g, _ = s.moments()
    assert max_rel(r_g, r_o) < 1e-10 and np.abs(U_g - U_o).max() < 1e-10
    sigma = 0.2
    lib = Wt.measure_column(r_g.reshape(ny, nx), nw, H, p, sigma)
    geo = WA.geometric_angle(r_o.reshape(ny, nx), nw, H, rl, rv)
    yl = WA.young_laplace_angle(fl.pressure(r_o.reshape(ny, nx)[ny // 2, nx // 2]),
                                fl.pressure(r_o.reshape(ny, nx)[ny // 2, 2]), sigma, H)
    assert abs(lib["theta_geom"] - geo) < 0.5 and abs(lib["theta_yl"] - yl) < 1e-6
    assert 110 < geo < 135


def test_calibration_in_the_h70_channel():
    import paper_2112_01975_amd as P
    from paper_2112_01975_amd import wetting as Wt
    base = _fluid(P, 0.7, 4.0, 0.725)
    rv, rl, _, _ = P.lbm_coexistence(base)
    sigma = Wt.effective_surface_tension(base, radius=24.0, n=96, steps=20000)
    assert 1.1 < sigma / P.lbm_surface_tension(base) < 1.3
    table = Wt.calibrate(base, [rv + f * (rl - rv) for f in (0.45, 0.5, 0.55, 0.6, 0.65)], H=70, wall=2,
                         nx=210, steps=60000, sigma=sigma)
    th = [t["theta_geom"] for t in table]
    assert all(a > b for a, b in zip(th, th[1:])) and th[0] > 85 and th[-1] < 62
    for t in table:
        assert abs(t["theta_geom"] - t["theta_yl"]) < 1.0
    for target in (59.3, 63.4):
        rw = Wt.wall_density_for_angle(table, target)
        got = Wt.column_angle(base, rw, 70, 2, 210, 60000, sigma=sigma)
        assert abs(got["theta_geom"] - target) < 0.5


def test_wettability_driven_column_matches_closed_form():
    import paper_2112_01975_amd as P
    from paper_2112_01975_amd import wetting as Wt
    from tests.golden_values import scalars
    g = scalars("wettability_column")
    W, nu = 4.0, g["nu"]
    base = _fluid(P, 0.7, W, 0.5 + 3 * nu)
    rv, rl, _, _ = P.lbm_coexistence(base)
    sigma = Wt.effective_surface_tension(base, radius=24.0, n=96, steps=20000)
    table = Wt.calibrate(base, [rv + f * (rl - rv) for f in (0.55, 0.6, 0.65, 0.7)], H=70, wall=2, nx=210,
                         steps=60000, sigma=sigma)
    th_m, th_p = g["theta_minus"], g["theta_plus"]
    rw_m, rw_p = Wt.wall_density_for_angle(table, th_m), Wt.wall_density_for_angle(table, th_p)
    H, Lx, Ll, nw = int(g["H"]), int(g["L"]), int(g["L_l"]), 2
    mask, rho0 = L.channel_column(Lx, H, nw, rl, rv, W, (Lx - Ll) / 2, (Lx + Ll) / 2)
    ny = H + 2 * nw
    p = replace(base, nx=Lx, ny=ny, mask=mask, rho_wall=rw_m)
    xs = np.arange(Lx)[None, :]

    def centroid(rho):
        w = np.clip(rho.reshape(ny, Lx)[nw:ny - nw] - rv, 0.0, None)
        return float((w * xs).sum() / w.sum())

    with P.Simulation(p) as s:                      # equal angles: the column stays put
        s.init(rho0)
        s.step(40000)
        rho, _, _ = s.moments()
        snap = P.lbm_get_populations(s.ctx)
    X0 = centroid(rho)
    assert abs(X0 - Lx / 2) < 0.1                  # symmetric about x = Lx / 2
    wall = np.where(np.arange(Lx)[None, :] >= Lx // 2, rw_p, rw_m) * np.ones((ny, 1))
    p2 = replace(p, rho_wall_field=wall.ravel())
    visc = rl * nu * Ll + rv * nu * (Lx - Ll)
    u_inf = sigma * H * (math.cos(math.radians(th_m)) - math.cos(math.radians(th_p))) / (6 * visc)
    t_inf = H * H * (rl * Ll + rv * (Lx - Ll)) / (12 * visc)
    xt = []
    with P.Simulation(p2) as s:                     # the right half turns less wettable
        s.init(rho0)
        P.lbm_set_populations(s.ctx, snap)
        for k in range(12):
            s.step(5000)
            rho, _, _ = s.moments()
            xt.append(X0 - centroid(rho))           # towards the more wettable (left) side
    t = 5000.0 * np.arange(1, 13)
    xa = t_inf * u_inf * (np.exp(-t / t_inf) + t / t_inf - 1)
    assert all(x > 0 for x in xt)
    u_late = (xt[-1] - xt[-5]) / 20000.0
    assert abs(u_late / u_inf - 1) < 0.15
    for x, a in zip(xt[2:], xa[2:]):
        assert abs(x / a - 1) < 0.2
