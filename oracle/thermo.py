"""Oracle thermodynamics of the non-ideal fluid, FP64.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this module;
it is used by tests/, by __graft_entry__.smoke() and by bench.py's CPU-baseline
leg. It shares no code with the HIP library.

Contents (paper sections cited per function):
  * equations of state: van der Waals, Peng-Robinson, Redlich-Kwong-Soave,
    Carnahan-Starling (Sec. 3.1, eqs vdWEoS, PREoS, RKSEoS, CSEos), with the
    critical temperature taken from the printed a(Tc, Pc), b(Tc, Pc) relations;
    and the two Shan-Chen equations of state of the sound-speed appendix (eqs SCeos,
    SC1, SC2) with the coupling G = G_c / T_reduced;
  * the Maxwell equal-area construction for the coexistence densities
    (Sec. 3.1, eq Maxwell_equal_area), evaluated by quadrature of its integral;
  * the flat-interface profile of the second-gradient fluid (Sec. 2.1,
    eq 2nd_grad_energy): (kappa/2) rho'^2 equals the excess grand potential
    density, which gives the surface tension sigma and the capillary
    coefficient kappa that yields a requested interface width W (Sec. 3.6,
    eq interface_W).
"""
from __future__ import annotations

import math
import warnings
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

VDW, PR, RKS, CS, IDEAL, SC1, SC2 = 0, 1, 2, 3, 4, 5, 6
EOS_NAMES = {VDW: "vdW", PR: "PR", RKS: "RKS", CS: "CS", IDEAL: "ideal", SC1: "SC-I", SC2: "SC-II"}

# Shan-Chen equations of state (appendix on the isothermal sound speed, eqs SCeos, SC1,
# SC2), read as P = rho/3 + (G/6) psi_SC(rho)^2: the classical form whose critical points
# are the ones the paper prints (the printed eq SCeos carries P0 = rho/3 in the second
# term as well, which moves the critical point away from both printed pairs).
#   SC-I : psi = 1 - exp(-rho),  d2P = 0 at exp(-rho) = 1/2, dP = 0 there at G = -4;
#   SC-II: psi = exp(-1/rho),    d2P = 0 at rho = 1,         dP = 0 there at G = -e^2.
# G enters as G = G_c / T_reduced, a pseudo-temperature with coexistence below T_r = 1.
SC_GC = {SC1: -4.0, SC2: -math.exp(2.0)}
SC_RHO_SEARCH = 50.0   # no repulsive pole: upper end of the density search


@dataclass(frozen=True)
class Fluid:
    """A non-ideal fluid: EOS kind, a, b, gas constant R, acentric factor and T/Tc."""
    eos: int
    a: float
    b: float
    T_reduced: float
    R: float = 1.0
    acentric: float = 0.0

    # -- critical temperature from the printed parameter relations (Sec. 3.1) --
    @property
    def Tc(self) -> float:
        a, b, R = self.a, self.b, self.R
        if self.eos == VDW:      # a = 27 R^2 Tc^2 / (64 Pc), b = R Tc / (8 Pc)
            return 8.0 * a / (27.0 * b * R)
        if self.eos == PR:       # a = 0.45724 R^2 Tc^2 / Pc, b = 0.0778 R Tc / Pc
            return 0.0778 * a / (0.45724 * b * R)
        if self.eos == RKS:      # a = 0.42748 R^2 Tc^2 / Pc, b = 0.08664 R Tc / Pc
            return 0.08664 * a / (0.42748 * b * R)
        if self.eos == CS:       # a = 0.4963 R^2 Tc^2 / Pc, b = 0.18727 R Tc / Pc
            return 0.18727 * a / (0.4963 * b * R)
        return 1.0 / 3.0         # ideal lattice gas and Shan-Chen: no temperature scale

    @property
    def G(self) -> float:
        """Shan-Chen coupling G = G_c / T_reduced (Shan-Chen kinds only)."""
        return SC_GC[self.eos] / self.T_reduced

    @property
    def T(self) -> float:
        return self.T_reduced * self.Tc

    @property
    def alpha(self) -> float:
        """Temperature factor alpha(T) of the PR and RKS attraction terms."""
        tr = self.T_reduced
        w = self.acentric
        if self.eos == PR:
            m = 0.37464 + 1.54226 * w - 0.26992 * w * w
        elif self.eos == RKS:
            m = 0.480 + 1.574 * w - 0.176 * w * w
        else:
            return 1.0
        return (1.0 + m * (1.0 - math.sqrt(tr))) ** 2

    @property
    def rho_max(self) -> float:
        """Upper end of the physical density range (repulsive pole)."""
        if self.eos in (VDW, PR, RKS):
            return 1.0 / self.b
        if self.eos == CS:
            return 4.0 / self.b
        if self.eos in (SC1, SC2):
            return SC_RHO_SEARCH
        return math.inf

    # -- the equation of state and its density derivative --
    def pressure(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        a, b, RT = self.a, self.b, self.R * self.T
        if self.eos == VDW:
            return rho * RT / (1.0 - b * rho) - a * rho * rho
        if self.eos == PR:
            return rho * RT / (1.0 - b * rho) - a * self.alpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho)
        if self.eos == RKS:
            return rho * RT / (1.0 - b * rho) - a * self.alpha * rho * rho / (1.0 + b * rho)
        if self.eos == CS:
            e = b * rho / 4.0
            return rho * RT * (1.0 + e + e * e - e ** 3) / (1.0 - e) ** 3 - a * rho * rho
        if self.eos == SC1:
            return rho / 3.0 + self.G / 6.0 * (1.0 - np.exp(-rho)) ** 2
        if self.eos == SC2:
            return rho / 3.0 + self.G / 6.0 * np.exp(-2.0 / rho)
        return rho / 3.0

    def dpressure(self, rho):
        """dP/drho, written out by hand for each EOS (isothermal sound speed squared)."""
        rho = np.asarray(rho, dtype=np.float64)
        a, b, RT = self.a, self.b, self.R * self.T
        if self.eos == VDW:
            return RT / (1.0 - b * rho) ** 2 - 2.0 * a * rho
        if self.eos == PR:
            q = 1.0 + 2.0 * b * rho - b * b * rho * rho
            dq = 2.0 * b - 2.0 * b * b * rho
            return RT / (1.0 - b * rho) ** 2 - a * self.alpha * (2.0 * rho * q - rho * rho * dq) / (q * q)
        if self.eos == RKS:
            q = 1.0 + b * rho
            return RT / (1.0 - b * rho) ** 2 - a * self.alpha * (2.0 * rho * q - rho * rho * b) / (q * q)
        if self.eos == CS:
            e = b * rho / 4.0
            num = 1.0 + e + e * e - e ** 3
            dnum = 1.0 + 2.0 * e - 3.0 * e * e
            den = (1.0 - e) ** 3
            # d/drho [rho num/den] with de/drho = b/4
            g = num / den + rho * (b / 4.0) * (dnum * den + 3.0 * num * (1.0 - e) ** 2) / (den * den)
            return RT * g - 2.0 * a * rho
        if self.eos == SC1:      # psi' = exp(-rho)
            return 1.0 / 3.0 + self.G / 3.0 * (1.0 - np.exp(-rho)) * np.exp(-rho)
        if self.eos == SC2:      # psi' = exp(-1/rho) / rho^2
            return 1.0 / 3.0 + self.G / 3.0 * np.exp(-2.0 / rho) / (rho * rho)
        return np.full_like(rho, 1.0 / 3.0)


# --------------------------------------------------------------------------------------------
# Maxwell equal-area construction (Sec. 3.1, eq Maxwell_equal_area)
# --------------------------------------------------------------------------------------------

def _bracket_roots(fun, lo, hi, n=20000, log=False):
    """Sign changes of fun on a grid over (lo, hi)."""
    xs = np.geomspace(lo, hi, n) if log else np.linspace(lo, hi, n)
    ys = fun(xs)
    idx = np.nonzero(np.sign(ys[:-1]) * np.sign(ys[1:]) < 0)[0]
    return [(xs[i], xs[i + 1]) for i in idx]


def spinodals(fl: Fluid):
    """Densities where dP/drho = 0 (the van der Waals loop's extrema), sorted."""
    hi = fl.rho_max * (1.0 - 1e-9)
    brs = _bracket_roots(fl.dpressure, hi * 1e-9, hi, log=True)
    roots = [optimize.brentq(lambda r: float(fl.dpressure(r)), lo_, hi_, xtol=1e-300, rtol=1e-15, maxiter=500)
             for lo_, hi_ in brs]
    if len(roots) != 2:
        raise ValueError(f"expected a van der Waals loop (2 spinodals) at T_r={fl.T_reduced}, got {roots}")
    return roots[0], roots[1]


def _branch_root(fl: Fluid, p, lo, hi):
    return optimize.brentq(lambda r: float(fl.pressure(r)) - p, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=1000)


def _area(fl: Fluid, psat, rv, rl):
    """Integral of (Psat - P)/rho^2 from rho_v to rho_l, in s = ln rho."""
    f = lambda s: (psat - float(fl.pressure(math.exp(s)))) * math.exp(-s)
    scale = abs(psat) * (1.0 / rv - 1.0 / rl)   # magnitude of either lobe
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(f, math.log(rv), math.log(rl), epsabs=1e-15 * scale, epsrel=2e-14, limit=1000)
    return val


def coexistence(fl: Fluid):
    """(rho_v, rho_l, P_sat) from the equal-area rule: P(rho_v) = P(rho_l) = P_sat and
    the integral of (P_sat - P)/rho^2 over [rho_v, rho_l] vanishes."""
    s_v, s_l = spinodals(fl)
    p_top = float(fl.pressure(s_v))
    p_bot = max(float(fl.pressure(s_l)), 0.0)
    tiny = 1e-300
    rmax = fl.rho_max * (1.0 - 1e-15)

    def roots(p):
        rv = _branch_root(fl, p, tiny, s_v)
        rl = _branch_root(fl, p, s_l, rmax)
        return rv, rl

    def g(p):
        rv, rl = roots(p)
        return _area(fl, p, rv, rl)

    span = p_top - p_bot
    lo = p_bot + 1e-14 * span if p_bot > 0 else p_top * 1e-30
    # g < 0 near p_top (vapour-side lobe dominates), g > 0 near the bottom
    psat = optimize.brentq(g, lo, p_top - 1e-13 * span, xtol=1e-300, rtol=1e-15, maxiter=2000)
    rv, rl = roots(psat)
    return rv, rl, psat


# --------------------------------------------------------------------------------------------
# Flat interface of the second-gradient fluid: sigma and kappa(W)
# --------------------------------------------------------------------------------------------

def excess_grand_potential(fl: Fluid, rho, rv, psat):
    """Omega(rho) - Omega_sat = rho * integral_{rho_v}^{rho} (P(s) - P_sat)/s^2 ds (>= 0 in the loop)."""
    f = lambda s: (float(fl.pressure(math.exp(s))) - psat) * math.exp(-s)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(f, math.log(rv), math.log(rho), epsabs=1e-15 * abs(psat) / rv,
                                epsrel=1e-13, limit=500)
    return rho * val


def max_excess(fl: Fluid):
    rv, rl, psat = coexistence(fl)
    res = optimize.minimize_scalar(lambda r: -excess_grand_potential(fl, r, rv, psat),
                                   bounds=(rv, rl), method="bounded",
                                   options={"xatol": 1e-12 * (rl - rv)})
    return -res.fun, res.x


def kappa_for_width(fl: Fluid, width: float) -> float:
    """Capillary coefficient for which the equilibrium profile has W = (rho_l - rho_v)/max|rho'|.

    From (kappa/2) rho'^2 = excess grand potential, max|rho'| = sqrt(2 max_excess / kappa).
    """
    rv, rl, _ = coexistence(fl)
    mx, _ = max_excess(fl)
    return 2.0 * mx * (width / (rl - rv)) ** 2


def interface_width(fl: Fluid, kappa: float) -> float:
    rv, rl, _ = coexistence(fl)
    mx, _ = max_excess(fl)
    return (rl - rv) / math.sqrt(2.0 * mx / kappa)


def surface_tension(fl: Fluid, kappa: float) -> float:
    """sigma = integral kappa rho'^2 dx = integral_{rho_v}^{rho_l} sqrt(2 kappa dOmega) drho."""
    rv, rl, psat = coexistence(fl)
    f = lambda r: math.sqrt(max(2.0 * kappa * excess_grand_potential(fl, r, rv, psat), 0.0))
    val, _ = integrate.quad(f, rv, rl, epsabs=0.0, epsrel=1e-10, limit=200)
    return val


def vdw_sigma_near_critical(fl: Fluid, kappa: float) -> float:
    """Near-critical van der Waals law sigma = 16a/(27 b^2) sqrt(kappa/a) (1 - T_r)^(3/2) (Sec. 3.2)."""
    return 16.0 * fl.a / (27.0 * fl.b ** 2) * math.sqrt(kappa / fl.a) * (1.0 - fl.T_reduced) ** 1.5


def vdw_critical_density(fl: Fluid) -> float:
    return 1.0 / (3.0 * fl.b)


def laplace_pressure_jump(sigma: float, radius: float, D: int) -> float:
    """Laplace's law with the equimolar radius (Sec. 3.2, eq Laplace_equimolar)."""
    return (D - 1) * sigma / radius


def equimolar_radius_2d(rho: np.ndarray, rho_v: float, rho_l: float) -> float:
    """Equimolar radius of a 2D drop from its mass adsorbance (Sec. 3.2, eq equmol2Ddrop),
    with the angular and radial integral taken as the sum over lattice nodes."""
    excess = float(np.sum(rho - rho_v))
    return math.sqrt(excess / (math.pi * (rho_l - rho_v)))


def equimolar_radius_3d(rho: np.ndarray, rho_v: float, rho_l: float) -> float:
    excess = float(np.sum(rho - rho_v))
    return (3.0 * excess / (4.0 * math.pi * (rho_l - rho_v))) ** (1.0 / 3.0)
