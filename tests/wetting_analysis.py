"""Test-side measurement of contact angles in the liquid-column channel (Sec. 4.5).

Used on oracle and GPU density fields alike; written independently of the
library's calibration module. A liquid column spans a channel of H fluid rows
between flat walls; at rest each meniscus is a circular arc.

- Geometric angle: the half-density crossings of the left meniscus, row by row
  away from the walls, fitted by a circle (algebraic least squares). The arc meets
  the walls, H apart, at |cos theta| = (H/2)/R; theta < 90 degrees when the centre
  lies on the vapour side (the liquid surface is concave).
- Young-Laplace angle: the bulk pressures inside and outside the column give the
  2D Laplace jump P_in - P_out = -2 sigma cos(theta) / H. The paper prints the law
  with sin(theta); that form vanishes at both 0 and 180 degrees, contradicting
  the limits the same section reports, so the cosine law is used.
"""
from __future__ import annotations

import math

import numpy as np


def meniscus_points(rho2d: np.ndarray, wall: int, rho_liquid: float, rho_vapour: float, skip: int = 3):
    """(x, y) of the half-density crossing of the left meniscus in every fluid row at least
    `skip` rows from a wall; the column is the liquid region around the middle in x."""
    ny, nx = rho2d.shape
    half = 0.5 * (rho_liquid + rho_vapour)
    pts = []
    for y in range(wall + skip, ny - wall - skip):
        row = rho2d[y]
        for x in range(nx // 2, 0, -1):
            a, b = row[x - 1] - half, row[x] - half
            if a * b <= 0 and a != b:
                pts.append((x - 1 + a / (a - b), float(y)))
                break
    return np.array(pts)


def circle_fit(pts: np.ndarray):
    """Centre (xc, yc) and radius of the circle x^2 + y^2 + D x + E y + F = 0 closest to the
    points in the algebraic least-squares sense."""
    A = np.stack([pts[:, 0], pts[:, 1], np.ones(len(pts))], 1)
    D, E, F = np.linalg.lstsq(A, -(pts[:, 0] ** 2 + pts[:, 1] ** 2), rcond=None)[0]
    xc, yc = -D / 2, -E / 2
    return xc, yc, math.sqrt(xc * xc + yc * yc - F)


def geometric_angle(rho2d, wall, H, rho_liquid, rho_vapour):
    pts = meniscus_points(rho2d, wall, rho_liquid, rho_vapour)
    xc, _, R = circle_fit(pts)
    c = min(1.0, 0.5 * H / R)
    wet = xc < pts[:, 0].mean()          # centre in the vapour to the left of the meniscus
    th = math.degrees(math.acos(c))
    return th if wet else 180.0 - th


def young_laplace_angle(p_in: float, p_out: float, sigma: float, H: int) -> float:
    c = -(p_in - p_out) * H / (2.0 * sigma)
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))
