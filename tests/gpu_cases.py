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

EOS_OF = {T.VDW: 0, T.PR: 1, T.RKS: 2, T.CS: 3, T.IDEAL: 4, T.SC1: 5, T.SC2: 6}


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
    accel: tuple = (0.0, 0.0, 0.0)
    rho_wall_field: np.ndarray | None = None
    link_q: np.ndarray | None = None    # [3,3(,3),N] wall fraction of the link n -> n + c, indexed by c + 1
    force_model: int = 0                # stencil coefficients of the force (Sec. 2.3.4), same codes both sides
    force_g: tuple = (0.0, 0.0, 0.0, 0.0)

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
                        self.T_reduced, self.kappa, self.tau, self.tau_vapour, rl, rv, self.rho_wall,
                        accel=self.accel, rho_wall_field=self.rho_wall_field, link_q=self.link_q,
                        force_model=self.force_model, force_g=self.force_g)

    def params(self, precision=0, rho_ref=0.0, check_every=0):
        import paper_2112_01975_amd as P
        rv, rl = self.coexistence() if self.eos != T.IDEAL else (1.0, 1.0)
        return P.Params(P.LBM_D3Q27 if self.lattice == 3 else P.LBM_D2Q9, self.nx, self.ny, self.nz,
                        EOS_OF[self.eos], self.a, self.b, 1.0, self.acentric, self.T_reduced, self.kappa,
                        self.tau, self.tau_vapour, rl, rv, self.rho_wall, self.mask, precision, rho_ref,
                        check_every, self.accel, self.rho_wall_field, self.library_link_q(),
                        force_model=self.force_model, force_g=self.force_g)

    def library_link_q(self):
        """link_q as the library takes it: [Q][N] in lbm_velocities order."""
        if self.link_q is None:
            return None
        import paper_2112_01975_amd as P
        cl = P.lbm_velocities(P.LBM_D3Q27 if self.lattice == 3 else P.LBM_D2Q9)
        cube = np.asarray(self.link_q, dtype=np.float64).reshape((3,) * self.lattice + (self.N,))
        return np.stack([cube[tuple(int(cl[i, a]) + 1 for a in range(self.lattice))] for i in range(len(cl))])


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


def oracle_one_step_at_nodes(case: Case, pops_bytes, precision, rho_ref, nodes, radius=6):
    """One oracle step on (2 radius + 1)^D neighbourhoods of sampled nodes of a GPU state.

    pops_bytes: lbm_get_populations of the GPU state at time t (Q rows of N values in the
    library's velocity order, post-collision values at the producing node). The physical
    pre-collision f_i(r) = row i at r - c_i (row opp(i) at r when r - c_i is solid), plus
    w_i rho_ref for FP32 deviation storage. Each neighbourhood is stepped once by the
    oracle on a periodic cube; with radius >= 6 the centre's rho and U at t + 1 depend on
    data inside the cube only. Returns [(rho, U[D])] per node.
    """
    import paper_2112_01975_amd as P
    D, nx, ny, nz, N = case.lattice, case.nx, case.ny, case.nz, case.N
    cl = P.lbm_velocities(P.LBM_D3Q27 if D == 3 else P.LBM_D2Q9)
    Q = len(cl)
    arr = np.frombuffer(pops_bytes, dtype=np.float64 if precision == 0 else np.float32).reshape(Q, N)  # no copy
    wcl = np.prod(np.where(cl[:, :D] == 0, 2.0 / 3.0, 1.0 / 6.0), axis=1)
    opp = np.array([int(np.nonzero((cl == -cl[i]).all(axis=1))[0][0]) for i in range(Q)])
    co, _, _ = O.lattice(D)
    to_lib = np.array([int(np.nonzero((cl == co[k]).all(axis=1))[0][0]) for k in range(Q)])
    mask = case.mask
    m = 2 * radius + 1
    out = []
    for (x0, y0, z0) in nodes:
        ox = (x0 + np.arange(-radius, radius + 1)) % nx
        oy = (y0 + np.arange(-radius, radius + 1)) % ny
        oz = (z0 + np.arange(-radius, radius + 1)) % nz if D == 3 else np.array([0])
        Z, Y, X = np.meshgrid(oz, oy, ox, indexing="ij")
        idx = (X + nx * (Y + ny * Z)).ravel()
        f = np.zeros((Q, idx.size))
        for i in range(Q):
            sx = (X - cl[i, 0]) % nx
            sy = (Y - cl[i, 1]) % ny
            sz = (Z - cl[i, 2]) % nz if D == 3 else Z
            src = (sx + nx * (sy + ny * sz)).ravel()
            vals = arr[i, src].astype(np.float64)
            if mask is not None:
                sol = mask[src].astype(bool)
                vals = np.where(sol, arr[opp[i], idx].astype(np.float64), vals)
            f[i] = vals + wcl[i] * rho_ref
        cube = Case(D, m, m, m if D == 3 else 1, case.eos, case.a, case.b, case.acentric, case.T_reduced,
                    case.kappa, case.tau, case.tau_vapour, case.rho_wall,
                    None if mask is None else mask[idx].copy(), case.accel,
                    None if case.rho_wall_field is None else case.rho_wall_field[idx].copy(),
                    force_model=case.force_model, force_g=case.force_g)
        cfg = cube.oracle_config()
        if case.tau_vapour > 0:
            rv, rl = case.coexistence()
            cfg.rho_vapour, cfg.rho_liquid = rv, rl
        o = O.Oracle(cfg, cube.mask)
        o.set_populations(f[to_lib])
        o.step(1)
        r, U, _ = o.moments()
        cidx = radius + m * (radius + m * (radius if D == 3 else 0))
        out.append((r[cidx], U[:, cidx]))
    return out
