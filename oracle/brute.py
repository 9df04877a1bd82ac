"""Independent vectorised NumPy step for tiny grids (pins lbm_oracle.c).

TEST INFRASTRUCTURE ONLY. Written separately from lbm_oracle.c in a different
style: populations live in a velocity cube indexed by (c_x+1, c_y+1[, c_z+1]),
shifts are np.roll over whole fields, streaming is written in pull form and the
product form (Sec. 2.3.2, eq prod) is an outer product of per-axis Psi triplets.
The equation of state comes from thermo.Fluid.

Step, with the readings used throughout the oracle: S = -F for the discrete
Korteweg force of eq Kforce_final (or its Shan-Chen, dual-range or general
stencil coefficients, Sec. 2.3.4), xi* = u + S/rho, zeta* = 1/3 + xi*^2 + Phi/rho,
Phi = (1 - omega/2) d_a(rho u_a^3) by central differences, halfway bounce-back,
or, when per-link wall distances are given, linearly interpolated bounce-back
(Bouzidi et al., the wall scheme cited in Sec. 4.5).
"""
from __future__ import annotations

import itertools

import numpy as np

from .thermo import Fluid

AXIS_W = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])   # Psi_{-1,0,+1}(0, 1/3)


def _stencil_pairs(model, kappa, g):
    """((G1, G2), (G3, G4)) of the pseudo-potential and capillary rings (Sec. 2.3.4)."""
    if model == 0:                       # eq Kforce_final
        return (4.0 / 3.0, -1.0 / 6.0), (2.0 * kappa, -kappa)
    if model == 1:                       # eq SCforce
        return (1.0, 0.0), (0.0, 0.0)
    if model == 2:                       # eq DRforce: eq PPcond1 only
        return (g[0], (1.0 - g[0]) / 2.0), (0.0, 0.0)
    return (g[0], g[1]), (g[2], g[3])


def _velocities(D):
    return list(itertools.product((-1, 0, 1), repeat=D))   # tuples (cx, cy[, cz])


def _psi_triplet(xi, zeta):
    """Stack [Psi_-1, Psi_0, Psi_+1](xi, zeta) along a new leading axis."""
    return np.stack([0.5 * (zeta - xi), 1.0 - zeta, 0.5 * (zeta + xi)])


def _cube(rho, xis, zetas):
    """rho * prod_a Psi_{c_a}(xi_a, zeta_a) as a (3,)*D + grid array."""
    trip = [_psi_triplet(x, z) for x, z in zip(xis, zetas)]
    if len(trip) == 2:
        return rho[None, None] * trip[0][:, None] * trip[1][None, :]
    return rho[None, None, None] * trip[0][:, None, None] * trip[1][None, :, None] * trip[2][None, None, :]


def _roll(field, c, k=1):
    """field(r + k c) for every r (periodic); grid axes are ordered (z, y, x) or (y, x)."""
    D = len(c)
    shifts = tuple(-k * c[a] for a in reversed(range(D)))
    return np.roll(field, shifts, axis=tuple(range(field.ndim - D, field.ndim)))


class BruteForce:
    """Tiny-grid FP64 reference: state f[(c)] on a grid of shape (ny, nx) or (nz, ny, nx)."""

    def __init__(self, D, shape, fluid: Fluid, kappa, tau, rho_wall=0.0, mask=None,
                 tau_vapour=0.0, rho_liquid=0.0, rho_vapour=0.0, accel=(0.0, 0.0, 0.0), rho_wall_field=None,
                 link_q=None, force_model=0, force_g=(0.0, 0.0, 0.0, 0.0)):
        self.D, self.shape = D, tuple(shape)
        self.fluid, self.kappa = fluid, kappa
        self.gpsi, self.grho = _stencil_pairs(force_model, kappa, force_g)
        self.tau, self.tau_v, self.rl, self.rv = tau, tau_vapour, rho_liquid, rho_vapour
        # per-node wall densities if given (only solid entries matter), else one value
        self.rho_wall = rho_wall if rho_wall_field is None else np.asarray(rho_wall_field, float).reshape(shape)
        self.accel = [float(g) for g in accel][:D]      # body-force acceleration: source + rho g
        self.solid = np.zeros(self.shape, bool) if mask is None else mask.reshape(self.shape).astype(bool)
        # link_q[(c)][r]: fraction of the link r -> r + c cut off by the wall (only links
        # from fluid into solid nodes matter); None means 1/2 everywhere
        self.link_q = None if link_q is None else np.asarray(link_q, float).reshape((3,) * D + self.shape)
        self.vel = _velocities(D)
        self.wcube = AXIS_W
        for _ in range(D - 1):
            self.wcube = np.multiply.outer(self.wcube, AXIS_W)

    def _idx(self, c):
        return tuple(ci + 1 for ci in c)

    def init(self, rho, U=None):
        """f = f_eq(rho, u) with u = U - S/(2 rho): U is the flow velocity (Appendix D)."""
        rho = rho.reshape(self.shape)
        U = np.zeros((self.D,) + self.shape) if U is None else U.reshape((self.D,) + self.shape)
        S = self._source(np.where(self.solid, self.rho_wall, rho))
        u = U - S / (2.0 * rho)
        self.f = _cube(rho, list(u), [1.0 / 3.0 + ua * ua for ua in u])
        self.f[(slice(None),) * self.D + (self.solid,)] = 0.0
        return self

    def _omega(self, rho):
        if self.tau_v <= 0.0:
            return np.full_like(rho, 1.0 / self.tau)
        nl, nv = (self.tau - 0.5) / 3.0, (self.tau_v - 0.5) / 3.0
        s = np.clip((rho - self.rv) / (self.rl - self.rv), 0.0, 1.0)
        return 1.0 / (3.0 * (nv + (nl - nv) * s) + 0.5)

    def _source(self, rho):
        """S = -F for eq Kforce_final plus the body force rho g, on a density field (solid
        nodes already hold rho_w)."""
        D = self.D
        P = self.fluid.pressure(rho)
        P0 = rho / 3.0
        psi = np.sqrt(np.abs(P - P0))
        sgn = np.where(P > P0, 1.0, -1.0)
        Fpsi = np.zeros((D,) + self.shape)
        Fcap = np.zeros((D,) + self.shape)
        for c in self.vel:
            w3 = 3.0 * self.wcube[self._idx(c)]
            tp = w3 * (self.gpsi[0] * _roll(psi, c, 1) + self.gpsi[1] * _roll(psi, c, 2))
            tc = w3 * (self.grho[0] * _roll(rho, c, 1) + self.grho[1] * _roll(rho, c, 2))
            for a in range(D):
                if c[a]:
                    Fpsi[a] += c[a] * tp
                    Fcap[a] += c[a] * tc
        F = 2.0 * sgn * psi * Fpsi + rho * Fcap
        S = -F + np.stack([rho * g for g in self.accel])
        return np.where(self.solid, 0.0, S)

    def fields(self):
        D = self.D
        vaxes = tuple(range(D))
        rho = self.f.sum(axis=vaxes)
        j = []
        for a in range(D):
            ca = np.array([-1.0, 0.0, 1.0]).reshape([3 if b == a else 1 for b in range(D)] + [1] * D)
            j.append((ca * self.f).sum(axis=vaxes))
        rho = np.where(self.solid, self.rho_wall, rho)
        u = np.stack([np.where(self.solid, 0.0, ja / rho) for ja in j])
        S = self._source(rho)
        return rho, u, S

    def step(self, n=1):
        D = self.D
        for _ in range(n):
            rho, u, S = self.fields()
            om = self._omega(rho)
            g = rho * u ** 3
            Phi = []
            for a in range(D):
                e = tuple(1 if b == a else 0 for b in range(D))
                Phi.append((1.0 - 0.5 * om) * 0.5 * (_roll(g[a], e, 1) - _roll(g[a], e, -1)))
            xs = [u[a] + S[a] / rho for a in range(D)]
            feq = _cube(rho, list(u), [1.0 / 3.0 + u[a] ** 2 for a in range(D)])
            fst = _cube(rho, xs, [1.0 / 3.0 + xs[a] ** 2 + Phi[a] / rho for a in range(D)])
            fpost = self.f + om * (feq - self.f) + (fst - feq)
            fnew = np.zeros_like(self.f)
            for c in self.vel:
                i = self._idx(c)
                ib = self._idx(tuple(-ci for ci in c))
                arrived = _roll(fpost[i], c, -1)            # value from r - c
                src_solid = _roll(self.solid, c, -1)
                back = fpost[ib]                            # halfway: reflected at r itself
                if self.link_q is not None:
                    # the wall cuts r -> r - c at q; pull back the value the interpolation
                    # places at r: from r and r + c (q < 1/2), or from both directions at r
                    q = self.link_q[ib]
                    behind = np.where(_roll(self.solid, c, 1), fpost[ib], _roll(fpost[ib], c, 1))
                    with np.errstate(divide="ignore", invalid="ignore"):
                        back = np.where(q < 0.5, 2.0 * q * fpost[ib] + (1.0 - 2.0 * q) * behind,
                                        fpost[ib] / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * fpost[i])
                fnew[i] = np.where(src_solid, back, arrived)
            fnew[(slice(None),) * D + (self.solid,)] = 0.0
            self.f = fnew
        return self

    def pressure_tensor(self):
        """Discrete pressure tensor of Appendix E on the whole grid, components xx, yy, [zz,]
        xy[, xz, yz] as a (D(D+1)/2, N) array: the lattice momentum flux of the pre-collision
        populations minus the four non-local parts (force = minus their divergence, momentum
        source = minus the force); zero at solid nodes."""
        D = self.D
        rho, _, _ = self.fields()
        P = self.fluid.pressure(rho)
        psi = np.sqrt(np.abs(P - rho / 3.0))
        sgn = np.where(P > rho / 3.0, 1.0, -1.0)
        pairs = [(0, 0), (1, 1), (0, 1)] if D == 2 else [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        out = []
        for a, b in pairs:
            flux = np.zeros(self.shape)
            ring1 = np.zeros(self.shape); ring2 = np.zeros(self.shape); across = np.zeros(self.shape)
            cap1 = np.zeros(self.shape); cap2 = np.zeros(self.shape); capx = np.zeros(self.shape)
            for c in self.vel:
                weight = 3.0 * np.prod([AXIS_W[ci + 1] for ci in c]) * c[a] * c[b]
                flux = flux + c[a] * c[b] * self.f[self._idx(c)]
                if weight == 0.0:
                    continue
                ring1 += weight * _roll(psi, c, 1)
                ring2 += weight * _roll(psi, c, 2)
                across += weight * _roll(psi, c, -1) * _roll(psi, c, 1)
                cap1 += weight * _roll(rho, c, 1)
                cap2 += weight * _roll(rho, c, 2)
                capx += weight * _roll(rho, c, -1) * _roll(rho, c, 1)
            (g1, g2), (g3, g4) = self.gpsi, self.grho
            nonlocal_ = (-sgn * g1 * psi * ring1 - sgn * g2 * (psi * ring2 + across)
                         - 0.5 * g3 * rho * cap1 - 0.5 * g4 * (rho * cap2 + capx))
            out.append(np.where(self.solid, 0.0, flux - nonlocal_).ravel())
        return np.stack(out)

    def moments(self):
        rho, u, S = self.fields()
        U = np.where(self.solid[None], 0.0, u + S / (2.0 * rho))
        return rho.ravel(), U.reshape(self.D, -1)
