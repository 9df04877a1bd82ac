"""Shared GPU-test case builders: one problem statement -> library Params and oracle Config.

Both sides receive the same seeded inputs from lbm_inputs; the coexistence
densities used to build profiles come from the oracle's thermodynamics.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import lbm_inputs as L
from oracle import oracle as O
from oracle import thermo as T

EOS_OF = {T.VDW: 0, T.PR: 1, T.RKS: 2, T.CS: 3, T.IDEAL: 4}


@dataclass
class Case:
    lattice: int            # 2 or 3
    nx: int
    ny: int
    nz: int = 1
    eos: int = T.VDW
    a: float = 9.0 / 49.0
    b: float = 2.0 / 21.0
    acentric: float = 0.0
    T_reduced: float = 0.9
    kappa: float = 0.02
    tau: float = 0.8
    tau_vapour: float = 0.0
    rho_wall: float = 0.0
    mask: np.ndarray | None = None

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def fluid(self):
        return T.Fluid(self.eos, self.a, self.b, self.T_reduced, 1.0, self.acentric)

    def coexistence(self):
        return T.coexistence(self.fluid())[:2]

    def oracle_config(self):
        rv, rl = self.coexistence() if self.eos != T.IDEAL else (1.0, 1.0)
        return O.Config(self.lattice, self.nx, self.ny, self.nz, self.eos, self.a, self.b, 1.0, self.acentric,
                        self.T_reduced, self.kappa, self.tau, self.tau_vapour, rl, rv, self.rho_wall)

    def params(self, precision=0, rho_ref=0.0, check_every=0):
        import paper_2112_01975_amd as P
        rv, rl = self.coexistence() if self.eos != T.IDEAL else (1.0, 1.0)
        return P.Params(P.LBM_D3Q27 if self.lattice == 3 else P.LBM_D2Q9, self.nx, self.ny, self.nz,
                        EOS_OF[self.eos], self.a, self.b, 1.0, self.acentric, self.T_reduced, self.kappa,
                        self.tau, self.tau_vapour, rl, rv, self.rho_wall, self.mask, precision, rho_ref,
                        check_every)


def run_oracle(case: Case, rho0, u0, steps):
    o = O.Oracle(case.oracle_config(), case.mask).init(rho0, u0)
    o.step(steps)
    return o.moments()


def run_gpu(case: Case, rho0, u0, steps, precision=0, rho_ref=0.0):
    import paper_2112_01975_amd as P
    with P.Simulation(case.params(precision, rho_ref)) as s:
        s.init(rho0, u0)
        if steps:
            s.step(steps)
        return s.moments()


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def slab_case_inputs(case: Case, width=4.0, noise=1e-4, seed=1001, axis=0):
    rv, rl = case.coexistence()
    rho = L.flat_slab(case.nx, case.ny, case.nz, rl, rv, width, axis=axis, noise=noise, seed=seed)
    return rho, None


def drop_case_inputs(case: Case, radius, width=5.0, noise=1e-5, seed=1003, centre=None):
    rv, rl = case.coexistence()
    rho = L.drop(case.nx, case.ny, case.nz, radius, rl, rv, width, centre=centre, noise=noise, seed=seed)
    return rho, None
