"""Closed-form solutions used as pins by the tests (no simulation code)."""
import numpy as np


def layered_poiseuille(y, H, h, g, ml, mv, rl, rv):
    """Steady layered Poiseuille flow (Sec. 4.2, eqs Poiseuille_odes with their boundary
    conditions; Appendix F): liquid 0 <= y <= h, vapour above, walls at y = 0 and H.
    b_l and c_v are the printed coefficients; b_v is the one that solves the printed system
    (the printed b_v lacks the term -h^2 mu_v rho_l in its numerator).
    Returns (u(y), (a_l, b_l, a_v, b_v, c_v))."""
    al, av = -rl * g / (2 * ml), -rv * g / (2 * mv)
    den = H * ml - h * ml + h * mv
    bl = g * (H * H * ml * rv - 2 * h * h * ml * rl + h * h * ml * rv + h * h * mv * rl + 2 * H * h * ml * rl
              - 2 * H * h * ml * rv) / (2 * ml * den)
    bv = g * (H * H * ml * rv - h * h * ml * rv - h * h * mv * rl + 2 * h * h * mv * rv) / (2 * mv * den)
    cv = g * H * (h * h * ml * rv + h * h * mv * rl - 2 * h * h * mv * rv - H * h * ml * rv + H * h * mv * rv) / (2 * mv * den)
    return np.where(y <= h, al * y * y + bl * y, av * y * y + bv * y + cv), (al, bl, av, bv, cv)
