"""D3Q27 parity over 1000 steps, through the single-pass (fused) step.

Bar: FP64 storage within 1e-10 of the oracle, node by node, in density (relative) and
flow velocity (absolute, lattice units) after 1000 steps (eq LBGK iterated); FP32
deviation storage against the same oracle state with the pointwise bound stated per
case. Three shapes of the 3D workloads:
  - the static drop (Peng-Robinson, T/Tc = 0.6, density ratio 853, W = 5, radius 16);
  - the drop impact on a pillar-textured floor (square pillars 8 wide, gap 8, 16 high,
    as in the 512 x 256 x 256 impact box), two viscosities nu_v = 15 nu_l with
    tau_liquid = 0.51 and 0.55, wall density = vapour density, drop radius 10 moving at
    -0.05 towards the pillars;
  - a drop impacting tapered posts whose wall links carry exact cut fractions (interpolated
    bounce-back), 48 x 48 x 40.
"""
import numpy as np
import pytest

import lbm_inputs as L
from oracle import thermo as T
from tests.gpu_cases import Case, max_rel, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

A_PR06 = 0.005046          # a for W = 5 at kappa 0.02, T/Tc 0.6, b = 2/21 (Peng-Robinson)
STEPS = 1000


def _drop():
    case = Case(3, 64, 64, 64, eos=T.PR, a=A_PR06, acentric=0.344, T_reduced=0.6, kappa=0.02, tau=0.8)
    rv, rl = case.coexistence()
    rho0 = L.drop(64, 64, 64, 16.0, rl, rv, 5.0, noise=1e-5, seed=1003)
    return case, rho0, None, rv


def _impact(tau):
    n = 64
    mask = L.pillar_mask(n, n, n, 8, 8, 16)
    fl = T.Fluid(T.PR, A_PR06, 2 / 21, 0.6, 1.0, 0.344)
    rv, rl, _ = T.coexistence(fl)
    case = Case(3, n, n, n, eos=T.PR, a=A_PR06, acentric=0.344, T_reduced=0.6, kappa=0.02, tau=tau,
                tau_vapour=0.5 + 15 * (tau - 0.5), rho_wall=rv, mask=mask)
    rho0 = L.drop(n, n, n, 10.0, rl, rv, 5.0, centre=(32.0, 32.0, 30.0), noise=1e-5, seed=1005)
    rho0 = np.where(mask.astype(bool), rv, rho0)
    u0 = L.impact_drop_velocity(rho0, rl, rv, 3, -0.05, 2)
    return case, rho0, u0, rv


def _check(case, rho0, u0, rv, fp32_rho_tol, fp32_u_tol):
    fluid = np.ones(case.N, bool) if case.mask is None else ~case.mask.astype(bool)
    r_o, U_o, t_o = run_oracle(case, rho0, u0, STEPS)
    assert np.all(np.isfinite(r_o)), "reference run diverged"
    r_g, U_g, t_g = run_gpu(case, rho0, u0, STEPS)
    err_r, err_u = max_rel(r_g, r_o), float(np.abs(U_g - U_o).max())
    print(f"FP64 after {STEPS} steps: max rel rho {err_r:.2e}, max |dU| {err_u:.2e}")
    assert err_r <= 1e-10 and err_u <= 1e-10
    assert abs(t_g[0] - t_o[0]) <= 1e-12 * t_o[0]
    r_f, U_f, t_f = run_gpu(case, rho0, u0, STEPS, precision=1, rho_ref=rv)
    ef_r = float(np.max(np.abs(r_f - r_o)[fluid] / r_o[fluid]))
    ef_u = float(np.abs(U_f - U_o).max())
    print(f"FP32 after {STEPS} steps: max rel rho {ef_r:.2e}, max |dU| {ef_u:.2e}, "
          f"mass drift {abs(t_f[0] / t_o[0] - 1):.2e}")
    assert ef_r <= fp32_rho_tol and ef_u <= fp32_u_tol
    assert abs(t_f[0] / t_o[0] - 1) <= 1e-6


def test_drop_64cubed_1000_steps():
    # FP32 bound: the liquid's populations keep ~7 digits of f - w rho_v; over 1000 steps the
    # pointwise difference (measured 1.1e-5 in density, 4e-7 in velocity) is stated at 1e-4 of
    # the local density and 1e-5 in velocity
    _check(*_drop(), 1e-4, 1e-5)


@pytest.mark.parametrize("tau", [0.51, 0.55])
def test_impact_on_pillars_64cubed_1000_steps(tau):
    # FP32 bound: largest at the drop's interface near the pillars, where the vapour side is a
    # thousandth of the liquid density (measured 7.0e-4 at tau_l = 0.51, 4.6e-4 at 0.55;
    # velocity 8e-6); stated bounds 2e-3 in density and 1e-4 in velocity
    _check(*_impact(tau), 2e-3, 1e-4)


def test_tapered_posts_interpolated_walls_1000_steps():
    # the interpolated-wall (Bouzidi) kernels over a long run: a drop impacting tapered posts
    # with exact cut fractions (48 x 48 x 40, two viscosities, tau_v = 1.25), 1000 steps, so that
    # the drop reaches and wets the posts; FP64 to the parity bar, FP32 to the stated bound
    from tests.test_gpu_walls import _posts_case
    case, rho0, u0, rv = _posts_case(48, 48, 40, 1.25)
    # FP32 measured: 6.5e-5 in density, 1.8e-6 in velocity; stated 2e-3 and 1e-4 as for the pillars
    _check(case, rho0, u0, rv, 2e-3, 1e-4)
