"""CPU pins of the host-side measurements in the wetting module (Sec. 4.5, Sec. 3.2) on
synthetic fields of known answer:
- a liquid column whose menisci are circular arcs meeting the walls at a prescribed angle,
  wetting and non-wetting: the meniscus fit returns the angle, and the Young-Laplace angle
  is the cosine law of the two bulk pressures (evaluated here by the oracle's EOS);
- the inverse calibration interpolates linearly in cos(theta) and refuses angles outside
  the table;
- the Kirkwood-Buff integral of flat interfaces whose P_nn - P_tt are Gaussians of known
  area, normal along x (2D) and z (3D).
"""
import math

import numpy as np
import pytest

from oracle import thermo as T

A9, B21 = 9 / 49, 2 / 21


def _column(theta_deg, H=40, wall=2, nx=140, x_apex=45.0, W=4.0, rl=6.5, rv=0.4):
    """Density of a liquid column between flat walls, menisci = arcs at contact angle theta."""
    ny = H + 2 * wall
    yc = (ny - 1) / 2.0
    R = (H / 2.0) / abs(math.cos(math.radians(theta_deg)))
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    xr = (nx - 1) - x                       # mirror image for the right meniscus
    if theta_deg < 90:                      # centre in the vapour: liquid outside the circle
        xc = x_apex - R
        d = lambda xx: np.hypot(xx - xc, y - yc) - R
    else:                                   # centre in the liquid: liquid inside the circle
        xc = x_apex + R
        d = lambda xx: R - np.hypot(xx - xc, y - yc)
    dist = np.minimum(d(x), d(xr))
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2.0 * dist / W)
    return rho, ny, nx


@pytest.mark.parametrize("theta", [55.0, 70.0, 110.0, 130.0])
def test_meniscus_fit_returns_the_contact_angle(theta):
    import paper_2112_01975_amd as P
    from paper_2112_01975_amd import wetting as Wt
    tr = 0.7
    p = P.Params(P.LBM_D2Q9, 8, 4, 1, P.LBM_EOS_VDW, A9, B21, 1.0, 0.0, tr, 0.02, 0.8)
    rv, rl, _, _ = P.lbm_coexistence(p)
    H, wall = 40, 2
    rho, ny, nx = _column(theta, H, wall, rl=rl, rv=rv)
    sigma = 0.2
    out = Wt.measure_column(rho, wall, H, p, sigma)
    assert abs(out["theta_geom"] - theta) < 0.3, out
    fl = T.Fluid(T.VDW, A9, B21, tr)
    dp = fl.pressure(rho[ny // 2, nx // 2]) - fl.pressure(rho[ny // 2, 2])
    c = max(-1.0, min(1.0, -dp * H / (2 * sigma)))
    assert abs(out["theta_yl"] - math.degrees(math.acos(c))) < 1e-9


def test_inverse_calibration_interpolates_in_cosine():
    from paper_2112_01975_amd import wetting as Wt
    # wall density linear in cos(theta): the interpolation is exact between the points
    table = [{"theta_geom": th, "rho_wall": 1.0 + 2.0 * math.cos(math.radians(th))} for th in (40, 60, 90, 120, 150)]
    for th in (45.0, 63.4, 100.0, 149.0):
        assert abs(Wt.wall_density_for_angle(table, th) - (1.0 + 2.0 * math.cos(math.radians(th)))) < 1e-12
    with pytest.raises(ValueError):
        Wt.wall_density_for_angle(table, 30.0)
    with pytest.raises(ValueError):
        Wt.wall_density_for_angle(table, 170.0)


@pytest.mark.parametrize("D", [2, 3])
def test_kirkwood_buff_integral_of_two_flat_interfaces(D):
    import paper_2112_01975_amd as P
    from paper_2112_01975_amd import wetting as Wt
    sigma, w, p0 = 0.17, 1.3, 0.05
    L = 96
    s = np.arange(L, dtype=np.float64)
    g = sigma / (math.sqrt(2 * math.pi) * w) * (np.exp(-0.5 * ((s - 24.3) / w) ** 2)
                                                + np.exp(-0.5 * ((s - 71.6) / w) ** 2))
    if D == 2:
        nx, ny, nz = L, 5, 1
        gx = np.broadcast_to(g[None, :], (ny, nx)).ravel()
        tensor = np.stack([np.full(nx * ny, p0), p0 - gx, np.zeros(nx * ny)])      # xx, yy, xy
        got = Wt.kirkwood_buff_integral(tensor, P.LBM_D2Q9, nx, ny, 1, axis=0)
    else:
        nx, ny, nz = 4, 3, L
        gz = np.broadcast_to(g[:, None, None], (nz, ny, nx)).ravel()
        N = nx * ny * nz
        # normal along z: P_zz uniform, P_xx and P_yy carry the deficit
        tensor = np.stack([p0 - gz, p0 - gz, np.full(N, p0), np.zeros(N), np.zeros(N), np.zeros(N)])
        got = Wt.kirkwood_buff_integral(tensor, P.LBM_D3Q27, nx, ny, nz, axis=2)
    # the node sum of a Gaussian of width 1.3 on a unit grid equals its area to ~1e-10
    assert abs(got / (2 * sigma) - 1) < 1e-8, got
