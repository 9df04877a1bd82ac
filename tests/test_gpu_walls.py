"""GPU parity of interpolated (Bouzidi) bounce-back against the FP64 oracle.

Walls that cut the links into solid nodes at a fraction q (Sec. 4.5, Sec. 5.3) run in
the two-pass step. Bar as in the other parity tests: FP64 storage within 1e-10 of the
oracle in density (relative) and velocity (absolute); FP32 deviation storage within the
tolerance stated per test.
"""
import math

import numpy as np
import pytest

import lbm_inputs as L
from oracle import thermo as T
from tests.gpu_cases import Case, max_rel, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FP64_RHO_TOL = 1e-10
FP64_U_TOL = 1e-10


def _cmp64(case, rho0, u0, steps):
    r_o, U_o, t_o = run_oracle(case, rho0, u0, steps)
    assert np.all(np.isfinite(r_o)) and np.all(np.isfinite(U_o)), "reference run diverged"
    r_g, U_g, t_g = run_gpu(case, rho0, u0, steps)
    err_r = max_rel(r_g, r_o)
    err_u = float(np.abs(U_g - U_o).max())
    assert err_r <= FP64_RHO_TOL, f"max rel rho error {err_r:.3e}"
    assert err_u <= FP64_U_TOL, f"max U error {err_u:.3e}"
    return r_o, U_o


def _random_walls(D, nx, ny, nz, seed, lo=0.05, hi=0.95):
    # q in [0.05, 0.95): both branches of the interpolation, and nodes cut on two opposite
    # links stay solvable at init (1/(2q) + 1/(2q') > 1.05)
    fl = T.Fluid(T.VDW, 0.02, 2 / 21, 0.8)
    rv, rl, _ = T.coexistence(fl)
    N = nx * ny * nz
    mask = L.random_mask(nx, ny, nz, 0.12, seed)
    case = Case(D, nx, ny, nz, a=0.02, T_reduced=0.8, rho_wall=0.5 * (rv + rl), mask=mask,
                link_q=L.random_link_q(D, N, lo, hi, seed + 1))
    rho0, u0 = L.random_state(N, D, rv, rl, 0.02, seed + 2)
    return case, rho0, u0, (rv, rl)


@pytest.mark.parametrize("walls", ["none", "halfway", "interpolated"])
@pytest.mark.parametrize("prec", [0, 1])
def test_d2q9_single_pass_matches_two_pass(walls, prec, monkeypatch):
    # The D2Q9 step in one pass (each tile's staged nodes pull their own populations for rho
    # and g) against the moment pass followed by the collide (LBM2P_TWO_PASS=1). Both passes
    # run the same per-node functions, but they are compiled into different kernels, whose
    # fused multiply-adds may round differently. The states therefore agree to rounding only.
    # The grid is ragged (37 x 29: partial tiles in x and y) and the run is 150 steps.
    # Bounds: FP64 1e-12 relative in density and 1e-12 absolute in U; FP32 1e-5 and 1e-6.
    import paper_2112_01975_amd as P
    case, rho0, u0, (rv, rl) = _random_walls(2, 37, 29, 1, 71)
    if walls == "none":
        case = Case(2, 37, 29, a=0.02, T_reduced=0.8)
    elif walls == "halfway":
        case = Case(2, 37, 29, a=0.02, T_reduced=0.8, rho_wall=case.rho_wall, mask=case.mask)
    out = {}
    for two in ("0", "1"):
        monkeypatch.setenv("LBM2P_TWO_PASS", two)
        with P.Simulation(case.params(prec, rv if prec else 0.0)) as s:
            s.init(rho0, u0).step(150)
            out[two] = (P.lbm_get_populations(s.ctx), s.moments())
    (r1, U1, t1), (r2, U2, t2) = out["0"][1], out["1"][1]
    assert np.all(np.isfinite(r1)) and np.all(np.isfinite(U1))
    er, eu = max_rel(r1, r2), float(np.abs(U1 - U2).max())
    print(f"{walls} prec {prec}: density {er:.2e}, U {eu:.2e}, bitwise {np.array_equal(out['0'][0], out['1'][0])}",
          flush=True)
    tr, tu = (1e-12, 1e-12) if prec == 0 else (1e-5, 1e-6)
    assert er < tr and eu < tu, (er, eu)
    assert abs(t1[0] - t2[0]) <= 1e-12 * abs(t2[0])


def test_interpolated_walls_random_q_d2q9_fp64():
    case, rho0, u0, _ = _random_walls(2, 37, 29, 1, 51)
    _cmp64(case, rho0, u0, 150)


def test_interpolated_walls_random_q_d3q27_fp64_and_fp32():
    # FP32 stated: density within 1e-4 relative and velocity within 1e-4 absolute of the
    # FP64 oracle after 60 steps (unit roundoff 6e-8 of deviations of order 1, amplified by
    # the random two-phase start)
    case, rho0, u0, (rv, rl) = _random_walls(3, 21, 14, 11, 61)
    r_o, U_o = _cmp64(case, rho0, u0, 60)
    r32, U32, _ = run_gpu(case, rho0, u0, 60, precision=1, rho_ref=rv)
    fl = ~case.mask.astype(bool)
    assert max_rel(r32[fl], r_o[fl]) < 1e-4
    assert np.abs(U32 - U_o).max() < 1e-4


def test_interpolated_walls_init_returns_inputs():
    # the init re-solves the wall slots so the interpolated pull returns the equilibria:
    # the moments of the initial state are the inputs, as for halfway bounce-back
    case, rho0, u0, _ = _random_walls(3, 13, 9, 7, 71)
    r_g, U_g, _ = run_gpu(case, rho0, u0, 0)
    r_o, U_o, _ = run_oracle(case, rho0, u0, 0)
    fl = ~case.mask.astype(bool)
    assert max_rel(r_g[fl], rho0[fl]) < 1e-13
    assert np.abs(U_g[:, fl] - u0[:, fl]).max() < 1e-13
    assert max_rel(r_g, r_o) < 1e-13 and np.abs(U_g - U_o).max() < 1e-13


@pytest.mark.parametrize("precision", [0, 1])
def test_interpolated_walls_at_half_equal_halfway_bitwise(precision, monkeypatch):
    # q = 1/2 everywhere gives interpolation weights 1 and 0: the same step bit for bit as
    # halfway bounce-back in the same (two-pass) kernels
    import paper_2112_01975_amd as P
    monkeypatch.setenv("LBM2P_TWO_PASS", "1")
    case, rho0, u0, (rv, _) = _random_walls(3, 19, 10, 9, 81)
    half = Case(**{**case.__dict__, "link_q": np.full_like(case.link_q, 0.5)})
    plain = Case(**{**case.__dict__, "link_q": None})
    out = []
    for c in (half, plain):
        with P.Simulation(c.params(precision, rv if precision else 0.0)) as s:
            s.init(rho0, u0)
            s.step(40)
            out.append(P.lbm_get_populations(s.ctx))
    assert np.array_equal(out[0], out[1])


def _frac_channel(D, nf, qb, qt, tau, g, nx=4, nz=3):
    """Ideal-gas channel driven along x: nf fluid rows between one solid row at each end,
    the walls cutting the links from the first and last fluid rows at qb and qt."""
    ny = nf + 2
    nz = nz if D == 3 else 1
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0] = 1
    mask[:, -1] = 1
    lq = np.zeros((3,) * D + (nz, ny, nx))
    lq[:, 0, ..., 1, :] = qb
    lq[:, 2, ..., ny - 2, :] = qt
    case = Case(D, nx, ny, nz, eos=T.IDEAL, a=0.0, b=0.0, T_reduced=1.0, kappa=0.0, tau=tau, rho_wall=1.0,
                mask=mask.ravel(), accel=(g, 0.0, 0.0), link_q=lq.reshape((3,) * D + (-1,)))
    H = (nf - 1) + qb + qt
    steps = int(30 * H * H / (math.pi ** 2 * (tau - 0.5) / 3))
    return case, np.ones(case.N), steps, H


@pytest.mark.parametrize("D", [2, 3])
def test_fractional_wall_poiseuille_fp64_and_fp32(D):
    # the oracle's second-order channel (walls at q = 0.25 and 0.75) run to steady state:
    # FP64 within 1e-10 of the oracle; FP32 (g = 1e-5, u_max 3.6e-3, deviations stored
    # to 6e-8) within 1e-3 of the peak velocity, and both on the parabola between the
    # true walls to the second-order wall offset of the scheme (< 2% of the peak here)
    tau, nf = 0.8, 16
    case, rho0, steps, H = _frac_channel(D, nf, 0.25, 0.75, tau, 1e-5)
    _, U_o = _cmp64(case, rho0, None, steps)
    _, U32, _ = run_gpu(case, rho0, None, steps, precision=1, rho_ref=1.0)
    nz = case.nz
    ux = U_o[0].reshape(nz, nf + 2, 4)[0, 1:-1, 0]
    ux32 = U32[0].reshape(nz, nf + 2, 4)[0, 1:-1, 0]
    y = np.arange(nf) + 0.25
    ua = 1e-5 * y * (H - y) / (2 * (tau - 0.5) / 3)
    assert np.abs(ux - ua).max() < 0.02 * ua.max()
    assert np.abs(ux32 - ux).max() < 1e-3 * ux.max()


def test_flow_past_a_sphere_d3q27_fp64_and_fp32():
    # body-force flow past a sphere of radius 4.3 off the lattice nodes: every link into it
    # carries its exact cut fraction (q from 0.014 to 1); two-phase vdW fluid at rest
    # density around the obstacle
    nx = ny = nz = 16
    mask, lq = L.sphere_obstacle(nx, ny, nz, (8.2, 7.7, 8.4), 4.3)
    fl = T.Fluid(T.VDW, 0.02, 2 / 21, 0.8)
    rv, rl, _ = T.coexistence(fl)
    case = Case(3, nx, ny, nz, a=0.02, T_reduced=0.8, tau=0.7, rho_wall=rl, mask=mask, accel=(1e-5, 0.0, 0.0),
                link_q=lq)
    rho0 = np.full(case.N, rl)
    r_o, U_o = _cmp64(case, rho0, None, 300)
    assert np.abs(U_o[0]).max() > 1e-4                      # a flow developed
    r32, U32, _ = run_gpu(case, rho0, None, 300, precision=1, rho_ref=rl)
    fl_ = ~mask.astype(bool)
    assert max_rel(r32[fl_], r_o[fl_]) < 1e-5
    assert np.abs(U32 - U_o).max() < 1e-3 * np.abs(U_o).max()


def _posts_case(nx, ny, nz, precision_tau_v=0.0):
    mask, lq = L.tapered_posts(nx, ny, nz, 2, 4.5, 2.0, 12.0, 16)
    case = Case(3, nx, ny, nz, eos=T.PR, a=0.005046, acentric=0.344, T_reduced=0.6, rho_wall=0.0102306,
                mask=mask, link_q=lq, tau_vapour=precision_tau_v)
    rv, rl = case.coexistence()
    rho0 = L.drop(nx, ny, nz, 10.0, rl, rv, 5.0, centre=(nx / 2, ny / 2, 26.0), noise=1e-5, seed=1009)
    rho0 = np.where(mask.astype(bool), rv, rho0)
    return case, rho0, L.impact_drop_velocity(rho0, rl, rv, 3, -0.05, 2), rv


@pytest.mark.parametrize("geometry", ["random", "posts"])
@pytest.mark.parametrize("precision", [0, 1])
def test_fused_interpolated_walls_match_two_pass(geometry, precision, monkeypatch):
    # the z-march with interpolated walls against the two-pass step on the same inputs:
    # random solids with random fractions on ragged tiles, and tapered posts with exact cut
    # fractions under an impacting drop; several z-chunks with a ragged last one. FP64:
    # the same arithmetic up to the order of a few sums; FP32 as the halfway comparison
    if geometry == "random":
        case, rho0, u0, (rv, _) = _random_walls(3, 48, 20, 36, 91)
    else:
        case, rho0, u0, rv = _posts_case(64, 32, 40, 1.25 if precision == 0 else 0.0)
    rr = rv if precision else 0.0
    monkeypatch.setenv("LBM2P_FUSED_TZ", "16")
    fused = run_gpu(case, rho0, u0, 30, precision=precision, rho_ref=rr)
    monkeypatch.setenv("LBM2P_TWO_PASS", "1")
    two = run_gpu(case, rho0, u0, 30, precision=precision, rho_ref=rr)
    assert np.all(np.isfinite(fused[0]))
    if precision == 0:
        assert max_rel(fused[0], two[0]) < 1e-12
        assert np.abs(fused[1] - two[1]).max() < 1e-13
    else:
        assert max_rel(fused[0], two[0]) < 1e-5
        assert np.abs(fused[1] - two[1]).max() < 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_tapered_posts_impact_fused_matches_oracle(precision):
    # the posts geometry through the default (fused) path against the oracle: FP64 to the
    # parity bar, FP32 density within 1e-5 and velocity within 1e-5 absolute after 40 steps
    case, rho0, u0, rv = _posts_case(32, 32, 40)
    r_o, U_o, _ = run_oracle(case, rho0, u0, 40)
    if precision == 0:
        r_g, U_g, _ = run_gpu(case, rho0, u0, 40)
        assert max_rel(r_g, r_o) <= FP64_RHO_TOL and np.abs(U_g - U_o).max() <= FP64_U_TOL
    else:
        r_g, U_g, _ = run_gpu(case, rho0, u0, 40, precision=1, rho_ref=rv)
        fl = ~case.mask.astype(bool)
        assert max_rel(r_g[fl], r_o[fl]) < 1e-5 and np.abs(U_g - U_o).max() < 1e-5
