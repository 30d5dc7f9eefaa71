"""Exact homogeneity of the GPU stage for the Euler equations.

Scaling the conserved state (averages and moments) by zeta leaves the
velocities, the sound speed and so the eigenvectors, the wave speeds and the
time step unchanged.  The characteristic variables and every point value,
flux and update then scale by zeta.  The smoothness indicators and u_ave
scale by zeta^2, and tau and beta_m u_ave by zeta^4.  So the weights of
Eq. (2.11)/(2.22) are unchanged when eps scales by zeta^4 as well: this is
the scale invariance the weights are designed for.  With zeta a power of two,
every rounding commutes with the scaling, so one step with the state scaled
by zeta and eps by zeta^4 must give exactly zeta times the unscaled step.

The check is GPU against GPU (no oracle arithmetic).  It covers both
precisions and both dimensions.  The weights are formed with one reciprocal
over products of the denominators beta_m u_ave + eps, which are first scaled
by a power of two so that the products do not follow the state's magnitude:
zeta = 2^200 puts the unscaled products of the five 2D denominators far
beyond the FP64 range (the state near 1e60, each denominator near 1e240).
The mixed form goes up to 2^60, where its FP32 point values and fluxes stay
clear of the FP32 overflow range, and down to 2^-40: at 2^-60 products of
small FP32 moment terms of the 2D form reach the subnormal range, where a
power of two no longer scales them exactly.
"""
import numpy as np
import pytest

import workloads as W
from oracle.driver import Problem

from gpu_util import gpu_three_stages, solver_for

pytestmark = pytest.mark.gpu

EPS = 1e-10


def _case(dim):
    if dim == 1:
        u, m = W.euler_1d_shocktube(1000, seed=3201)
        return Problem(1, "euler", 1000, (0, 1), bc="transmissive"), u, m
    u, m = W.euler_2d_vortex_quadrant(70, 64, seed=3200, q=2)
    return Problem(2, "euler", (70, 64), (0, 10, 0, 10)), u, m


CASES = ([("fp64", k) for k in (-200, -100, -40, -20, 20, 40, 100, 200)] +
         [("mixed", k) for k in (-40, -20, 20, 40, 60)])


@pytest.mark.parametrize("precision,k", CASES)
@pytest.mark.parametrize("dim", [1, 2])
def test_stage_is_homogeneous_under_power_of_two_scaling(dim, precision, k):
    P, u, m = _case(dim)
    if precision == "mixed":
        # the mixed form stores the moments in FP32: start from values that
        # are exact there, so that both runs see the same inputs
        m = m.astype(np.float32).astype(np.float64)
    zeta = 2.0 ** k
    alpha = P.max_wavespeed(u)
    dt = P.dt_from(alpha, 0.6)
    print(f"[gpu] homogeneity dim={dim} {precision} zeta=2^{k}", flush=True)
    S1 = solver_for(P, precision=precision)
    base = gpu_three_stages(S1, P, u, m, dt, alpha)
    S1.close()
    S2 = solver_for(P, precision=precision, eps=EPS * zeta ** 4)
    scaled = gpu_three_stages(S2, P, zeta * u, zeta * m, dt, alpha)
    S2.close()
    for s in range(3):
        for a, b, what in ((base[s][0], scaled[s][0], "averages"),
                           (base[s][1], scaled[s][1], "moments")):
            assert np.all(np.isfinite(b)), (dim, precision, k, s, what)
            diff = np.abs(zeta * a - b).max()
            assert diff == 0.0, (dim, precision, k, s, what, diff, np.abs(b).max())
