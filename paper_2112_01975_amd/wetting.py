"""Contact-angle calibration of the virtual wall density (Sec. 4.5), run on the GPU path.

Solid nodes carry a virtual density rho_w, which enters the pseudo-potential and the
capillary stencil of the neighbouring fluid nodes (after Benzi et al.); rho_w is the
one parameter that sets the equilibrium contact angle, from 180 degrees at rho_w =
rho_v to 0 at rho_w = rho_l. The paper maps it with a liquid column in a channel
(Young-Laplace test). This module reproduces that measurement through the library:

- effective_surface_tension: Laplace's law on a free 2D drop, sigma = (P_in - P_out) R
  with the equimolar radius; the model's sigma differs from the thermodynamic integral
  (lbm_surface_tension) by a discretisation factor that depends on the interface width.
- column_angle: a liquid column across a channel of H fluid rows between flat walls of
  density rho_w, stepped to rest; the angle from the meniscus (a circle fitted to the
  half-density crossings by geometric least squares) and from the pressure jump through
  the 2D Young-Laplace law P_in - P_out = -2 sigma cos(theta) / H.
- calibrate / wall_density_for_angle: the angle as a function of rho_w over a list of
  densities, and its inverse by interpolation in cos(theta).
- kirkwood_buff_integral: the surface tension of flat interfaces from the discrete
  pressure tensor (lbm_pressure_tensor), a second measure beside Laplace's law.

The paper prints the Young-Laplace law with sin(theta); that form vanishes at both ends
of the angle range it reports, so the cosine law is used here.
"""
from __future__ import annotations

import math
from dataclasses import replace

import numpy as np

from . import lbm as P


def _tanh(d, rl, rv, width):
    return 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2.0 * d / width)


def effective_surface_tension(base: P.Params, radius: float = 24.0, n: int = 96, steps: int = 20000,
                              width: float = 4.0) -> float:
    """Laplace's law on a periodic n x n D2Q9 drop of the given radius (base supplies the
    fluid: EOS, temperature, kappa, tau, precision); returns (P_in - P_out) * R_equimolar."""
    rv, rl, _, _ = P.lbm_coexistence(base)
    p = replace(base, lattice=P.LBM_D2Q9, nx=n, ny=n, nz=1, mask=None, rho_wall_field=None, link_q=None,
                accel=(0.0, 0.0, 0.0), rho_ref=rv if base.precision == P.LBM_FP32_DEV else 0.0)
    y, x = np.mgrid[0:n, 0:n]
    rho0 = _tanh(radius - np.hypot(x - n / 2, y - n / 2), rl, rv, width).ravel()
    with P.Simulation(p) as s:
        s.init(rho0)
        s.step(steps)
        rho, _, _ = s.moments()
    r2 = rho.reshape(n, n)
    rin, rout = float(r2[n // 2, n // 2]), float(r2[0, 0])
    re = math.sqrt(float(np.sum(rho - rout)) / (math.pi * (rin - rout)))
    pin, pout = P.lbm_eos_pressure(p, np.array([rin, rout]))
    return float((pin - pout) * re)


def _meniscus(rho2d, wall, rl, rv, skip):
    ny, nx = rho2d.shape
    half = 0.5 * (rl + rv)
    ys = np.arange(wall + skip, ny - wall - skip)
    xs = []
    for y in ys:
        row = rho2d[y, : nx // 2 + 1] - half
        k = np.nonzero(np.sign(row[:-1]) != np.sign(row[1:]))[0]
        if len(k) == 0:
            return None
        j = k[-1]                                  # last crossing left of the middle
        xs.append(j + row[j] / (row[j] - row[j + 1]))
    return np.array(xs), ys.astype(np.float64)


def _fit_circle(x, y):
    """Geometric least squares (Gauss-Newton on the distances to the circle), started from
    the centre straight off the meniscus at the largest distance implied by its bow."""
    yc = 0.5 * (y[0] + y[-1])
    mid = x[np.argmin(np.abs(y - yc))]
    bow = 0.5 * (x[0] + x[-1]) - mid
    half = 0.5 * (y[-1] - y[0])
    R = (half * half + bow * bow) / (2.0 * abs(bow)) if abs(bow) > 1e-9 else 1e6
    xc = mid + (R if bow > 0 else -R)
    for _ in range(50):
        dx, dy = x - xc, y - yc
        d = np.hypot(dx, dy)
        res = d - R
        J = np.stack([-dx / d, -dy / d, -np.ones_like(d)], 1)
        step = np.linalg.lstsq(J, -res, rcond=None)[0]
        xc, yc, R = xc + step[0], yc + step[1], R + step[2]
        if np.abs(step).max() < 1e-12 * max(1.0, abs(R)):
            break
    return xc, yc, abs(R)


def measure_column(rho2d: np.ndarray, wall: int, H: int, params: P.Params, sigma: float, skip: int = 3):
    """Angles of the column state rho2d ([ny, nx], liquid column in the middle of x)."""
    rv, rl, _, _ = P.lbm_coexistence(params)
    ny, nx = rho2d.shape
    pin, pout = P.lbm_eos_pressure(params, np.array([rho2d[ny // 2, nx // 2], rho2d[ny // 2, 2]]))
    dp = float(pin - pout)
    c_yl = max(-1.0, min(1.0, -dp * H / (2.0 * sigma)))
    out = {"dp": dp, "theta_yl": math.degrees(math.acos(c_yl))}
    m = _meniscus(rho2d, wall, rl, rv, skip)
    if m is None:
        out.update(theta_geom=float("nan"), radius=float("nan"))
        return out
    x, y = m
    xc, _, R = _fit_circle(x, y)
    th = math.degrees(math.acos(min(1.0, 0.5 * H / R)))
    wet = xc < x.mean()                           # centre on the vapour side: concave liquid
    out.update(theta_geom=th if wet else 180.0 - th, radius=R)
    return out


def column_angle(base: P.Params, rho_wall: float, H: int, wall: int = 2, nx: int | None = None,
                 steps: int = 20000, sigma: float | None = None, width: float = 4.0) -> dict:
    """One Young-Laplace column: H fluid rows between `wall` solid rows of density rho_wall,
    periodic length nx (default 3 H), liquid in the middle third; stepped `steps` times."""
    nx = nx or 3 * H
    ny = H + 2 * wall
    rv, rl, _, _ = P.lbm_coexistence(base)
    y, x = np.mgrid[0:ny, 0:nx]
    solid = (y < wall) | (y >= ny - wall)
    rho0 = np.where(solid, rv, _tanh(np.minimum(x - nx / 3, 2 * nx / 3 - x), rl, rv, width)).ravel()
    p = replace(base, lattice=P.LBM_D2Q9, nx=nx, ny=ny, nz=1, mask=solid.astype(np.uint8).ravel(), rho_wall=rho_wall,
                rho_wall_field=None, link_q=None, accel=(0.0, 0.0, 0.0),
                rho_ref=rv if base.precision == P.LBM_FP32_DEV else 0.0)
    if sigma is None:
        sigma = effective_surface_tension(base, width=width)
    with P.Simulation(p) as s:
        s.init(rho0)
        s.step(steps)
        rho, _, _ = s.moments()
    out = measure_column(rho.reshape(ny, nx), wall, H, p, sigma)
    out.update(rho_wall=rho_wall, sigma=sigma)
    return out


def calibrate(base: P.Params, rho_walls, H: int = 40, **kw) -> list[dict]:
    """column_angle for every wall density in rho_walls (one drop measures sigma first)."""
    sigma = kw.pop("sigma", None)
    if sigma is None:
        sigma = effective_surface_tension(base, width=kw.get("width", 4.0))
    return [column_angle(base, float(r), H, sigma=sigma, **kw) for r in rho_walls]


def kirkwood_buff_integral(tensor: np.ndarray, lattice: int, nx: int, ny: int, nz: int = 1, axis: int = 0) -> float:
    """Integral of P_nn - P_tt along the normal `axis` of flat interfaces (Kirkwood-Buff,
    Sec. 3.2), from lbm_pressure_tensor's output, averaged over the transverse nodes and
    tangential directions: the surface tension summed over the interfaces crossed."""
    D = 3 if lattice == P.LBM_D3Q27 else 2
    shape = (nz, ny, nx) if D == 3 else (ny, nx)
    diag = [tensor[a].reshape(shape) for a in range(D)]
    ax = D - 1 - axis                                        # array axis of the normal direction
    tang = [diag[a] for a in range(D) if a != axis]
    diff = diag[axis] - sum(tang) / len(tang)
    other = tuple(k for k in range(D) if k != ax)
    return float(diff.mean(axis=other).sum())


def wall_density_for_angle(table: list[dict], theta: float, key: str = "theta_geom") -> float:
    """Wall density giving the angle theta (degrees), interpolated linearly in cos(theta)
    between the calibration points (which must be monotone in rho_w)."""
    pts = sorted((math.cos(math.radians(t[key])), t["rho_wall"]) for t in table if np.isfinite(t[key]))
    c = math.cos(math.radians(theta))
    cs, rs = zip(*pts)
    if not (cs[0] <= c <= cs[-1]):
        raise ValueError("angle outside the calibrated range")
    return float(np.interp(c, cs, rs))
