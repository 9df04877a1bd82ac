"""Curvature-dependent surface tension of drops and bubbles (Sec. 3.4), from the discrete
pressure tensor (Appendix E) that lbm_pressure_tensor computes on the GPU.

- notional_surface_tension: sigma(R) of a dividing circle or sphere of radius R (eq sigmaR):
  the integral over r of (r/R)^(D-1) [P_perp(r, R) - P_par(r)], with P_par the tangential
  component of the discrete tensor and P_perp the normal pressure of the sharp-interface
  system. The printed P_perp puts the step with the opposite sign, which would not give
  P_out outside the dividing surface; it is read as P_in for r < R and P_out beyond.
  Over the lattice, r^(D-1) dr is the node volume over the area S_D of the unit sphere
  (S_2 = 2 pi, S_3 = 4 pi), and the step of P_perp integrates in closed form, so
      sigma(R) = sum_nodes (P_out - P_par) / (S_D R^(D-1)) + (P_in - P_out) R / D.
- fit_surface_of_tension: sigma_s and R_s from sigma(R) probes by least squares on eq
  surface_of_tension_drop, sigma(R) / sigma_s = (1/D)(R_s/R)^(D-1) + ((D-1)/D)(R/R_s),
  which is linear in the two functions R^(1-D) and R.
- equimolar_radius: R_e from zero mass adsorbance (eq equmol2Ddrop; in 3D the same
  condition on the sphere).
- tolman_length: delta_T from (R_s, sigma_s) of several drops or bubbles by least squares
  on eq tolman_length, sigma_s = sigma_0 (1 -+ (D-1) delta_T / R_s).

Host-side analysis of arrays the library returns (numpy only).
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm as P

_SPHERE = {2: 2.0 * math.pi, 3: 4.0 * math.pi}


def _dims_of(lattice: int):
    return 3 if lattice == P.LBM_D3Q27 else 2


def tangential_pressure(tensor: np.ndarray, lattice: int, nx: int, ny: int, nz: int = 1, centre=None):
    """Distance r from `centre` (default: the box centre, (n - 1)/2 per axis) and the
    tangential pressure per node, from lbm_pressure_tensor's output [D(D+1)/2][N]
    (components xx, yy, xy in 2D; xx, yy, zz, xy, xz, yz in 3D). In 3D the tangential
    pressure is the mean over the plane normal to the radius, (tr P - P_rr) / 2; at r = 0
    it is tr P / D. Offsets from the centre are taken without periodic wrapping: the drop or
    bubble must not cross the box boundary."""
    D = _dims_of(lattice)
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    shape = (nz, ny, nx) if D == 3 else (ny, nx)
    axes = [np.arange(n, dtype=np.float64) - c for n, c in zip((nx, ny, nz)[:D], centre[:D])]
    grids = np.meshgrid(*reversed(axes), indexing="ij")          # arrays indexed [z,] y, x
    d = [g.ravel() for g in reversed(grids)]                      # offsets along x, y[, z]
    r2 = sum(v * v for v in d)
    r = np.sqrt(r2)
    comp = [np.asarray(tensor[k], dtype=np.float64).reshape(-1) for k in range(D * (D + 1) // 2)]
    if comp[0].size != int(np.prod(shape)):
        raise ValueError("tensor size does not match the lattice dimensions")
    diag = comp[:D]
    off = {(0, 1): comp[D]} if D == 2 else {(0, 1): comp[3], (0, 2): comp[4], (1, 2): comp[5]}
    trace = sum(diag)
    with np.errstate(invalid="ignore", divide="ignore"):
        prr = sum(diag[a] * d[a] * d[a] for a in range(D))
        for (a, b), v in off.items():
            prr = prr + 2.0 * v * d[a] * d[b]
        prr = prr / r2
    ptt = (trace - prr) / (D - 1)
    ptt = np.where(r2 > 0, ptt, trace / D)
    return r, ptt


def notional_surface_tension(tensor: np.ndarray, lattice: int, nx: int, ny: int, nz: int, radii,
                             p_in: float, p_out: float, centre=None) -> np.ndarray:
    """sigma(R) for each R in radii (eq sigmaR) of a drop or bubble centred at `centre`,
    with bulk pressures p_in inside and p_out outside."""
    D = _dims_of(lattice)
    _, ptt = tangential_pressure(tensor, lattice, nx, ny, nz, centre)
    excess = float(np.sum(p_out - ptt))
    R = np.asarray(radii, dtype=np.float64)
    return excess / (_SPHERE[D] * R ** (D - 1)) + (p_in - p_out) * R / D


def fit_surface_of_tension(radii, sigma, D: int):
    """(sigma_s, R_s) of eq surface_of_tension_drop fitted to the probes sigma(radii):
    sigma(R) = alpha R^(1-D) + beta R with alpha = sigma_s R_s^(D-1) / D and
    beta = (D-1) sigma_s / (D R_s)."""
    R = np.asarray(radii, dtype=np.float64)
    A = np.stack([R ** (1 - D), R], axis=1)
    (alpha, beta), *_ = np.linalg.lstsq(A, np.asarray(sigma, dtype=np.float64), rcond=None)
    if alpha * beta <= 0:
        raise ValueError("the probes do not have the shape of a drop or bubble (alpha * beta <= 0)")
    # alpha / beta = R_s^D / (D - 1)
    rs = ((D - 1) * alpha / beta) ** (1.0 / D)
    return float(D * beta * rs / (D - 1)), float(rs)


def equimolar_radius(rho: np.ndarray, D: int, rho_in: float, rho_out: float) -> float:
    """Radius of the dividing circle (D = 2) or sphere (D = 3) of zero mass adsorbance for a
    drop (rho_in > rho_out) or bubble (rho_in < rho_out): the excess mass over the outside
    density equals that of a sharp body of density rho_in."""
    excess = float(np.sum(np.asarray(rho, dtype=np.float64) - rho_out)) / (rho_in - rho_out)
    if excess <= 0:
        raise ValueError("no excess of the inside phase")
    return math.sqrt(excess / math.pi) if D == 2 else (3.0 * excess / (4.0 * math.pi)) ** (1.0 / 3.0)


def tolman_length(rs, sigma_s, sigma_0: float, D: int, bubble: bool = False) -> float:
    """delta_T of eq tolman_length fitted by least squares (through the origin in 1/R_s) to
    the surfaces of tension of several drops (or bubbles)."""
    x = 1.0 / np.asarray(rs, dtype=np.float64)
    y = np.asarray(sigma_s, dtype=np.float64) / sigma_0 - 1.0
    slope = float(np.dot(x, y) / np.dot(x, x))          # y = -+ (D-1) delta x
    return (slope if bubble else -slope) / (D - 1)
