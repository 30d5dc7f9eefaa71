"""GPU parity: the HIP stage kernels (through the C-ABI) against the CPU
oracle on the same seeded inputs.

Tolerances (FP64 path): relative L-infinity per array <= 1e-12 after one
stage, <= 1e-10 after 100 steps.  The mixed path (FP32 moments, point values
and fluxes; FP64 averages, smoothness indicators and weights) is compared
with the FP64 oracle at the tolerances written in each test.
"""
import numpy as np
import pytest

import workloads as W
from oracle.driver import Problem

from gpu_util import (gpu_three_stages, oracle_three_stages, solver_for, state_err, to_gpu,
                      flat, unflat, rel_err)

pytestmark = pytest.mark.gpu

TOL_STAGE = 1e-12
TOL_STEPS = 1e-10


def _cases():
    """(name, Problem, u0, m0) -- sizes spanning several tiles/strips with
    ragged tails."""
    out = []
    u, m = W.advection_sine_1d(200)
    out.append(("adv1d_sine_200", Problem(1, "advection", 200, (0, 2), adv=(1.0,)), u, m))
    u, m = W.burgers_1d_initial(157)
    out.append(("burgers1d_157", Problem(1, "burgers", 157, (0, 2)), u, m))
    u, m = W.euler_1d_shocktube(1000, seed=2001)
    out.append(("euler1d_tube_1000", Problem(1, "euler", 1000, (0, 1), bc="transmissive"), u, m))
    u, m = W.random_smooth_1d(300, 3, seed=2002, positive_euler=True)
    out.append(("euler1d_smooth_300_comp",
                Problem(1, "euler", 300, (0, 2), char_decomp=False), u, m))
    u, m = W.burgers_2d_initial(70)
    out.append(("burgers2d_70", Problem(2, "burgers", (70, 70), (0, 4, 0, 4)), u, m))
    u, m = W.cell_moments_2d(lambda X, Y: np.sin(np.pi * X) * np.cos(np.pi * Y) + 0.3,
                             (0, 2, 0, 2), 131, 45)
    out.append(("adv2d_131x45", Problem(2, "advection", (131, 45), (0, 2, 0, 2),
                                        adv=(1.0, -0.5)), u, m))
    u, m = W.euler_2d_vortex_quadrant(130, 96, seed=3001, q=2)
    out.append(("euler2d_quad_130x96", Problem(2, "euler", (130, 96), (0, 10, 0, 10)), u, m))
    u, m = W.euler_2d_vortex_quadrant(70, 64, seed=3002, q=2)
    out.append(("euler2d_quad_70x64_trans",
                Problem(2, "euler", (70, 64), (0, 10, 0, 10),
                        bc=("transmissive", "periodic", "transmissive", "transmissive")), u, m))
    u, m = W.euler_2d_vortex_quadrant(64, 64, seed=3003, q=2)
    out.append(("euler2d_quad_64_comp",
                Problem(2, "euler", (64, 64), (0, 10, 0, 10), char_decomp=False), u, m))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_one_stage_fp64(case):
    name, P, u0, m0 = case
    print(f"[gpu] one-stage parity {name}", flush=True)
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    ref = oracle_three_stages(P, u0, m0, dt, alpha)
    S = solver_for(P)
    got = gpu_three_stages(S, P, u0, m0, dt, alpha, inputs=ref[:2])
    for s in range(3):
        eu, em = state_err(P, got[s], ref[s])
        assert eu <= TOL_STAGE and em <= TOL_STAGE, (name, s, eu, em)
    S.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[0] in
                                  ("adv1d_sine_200", "euler1d_tube_1000", "burgers2d_70",
                                   "euler2d_quad_70x64_trans")],
                         ids=lambda c: c[0])
def test_100_steps_fp64(case):
    import torch
    name, P, u0, m0 = case
    print(f"[gpu] 100-step parity {name}", flush=True)
    uo, mo, t, steps = P.advance(u0, m0, cfl=0.6, max_steps=100)
    S = solver_for(P)
    uf, mf = flat(P, u0, m0)
    ug, mg = to_gpu(uf), to_gpu(mf)
    tg, sg = S.advance(ug, mg, 0.6, 1e30, 100)
    torch.cuda.synchronize()
    assert sg == [100] and abs(tg[0] - t) <= 1e-12 * t
    got = unflat(P, ug.cpu().numpy(), mg.cpu().numpy())
    eu, em = state_err(P, got, (uo, mo))
    assert eu <= TOL_STEPS and em <= TOL_STEPS, (name, eu, em)
    S.close()


def test_advection_to_final_time_matches_oracle():
    """The sine-advection workload run to T = 2 at CFL 0.2 (1000 steps)."""
    import torch
    P = Problem(1, "advection", 200, (0, 2), adv=(1.0,))
    u0, m0 = W.advection_sine_1d(200)
    uo, mo, t, steps = P.advance(u0, m0, cfl=0.2, t_final=2.0)
    S = solver_for(P)
    ug, mg = to_gpu(u0), to_gpu(m0)
    tg, sg = S.advance(ug, mg, 0.2, 2.0, 10 ** 6)
    torch.cuda.synchronize()
    assert sg == [steps] == [1000] and abs(tg[0] - 2.0) < 1e-13
    eu, em = state_err(P, (ug.cpu().numpy(), mg.cpu().numpy()), (uo, mo))
    assert eu <= TOL_STEPS and em <= TOL_STEPS
    S.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[0] in
                                  ("euler1d_tube_1000", "euler2d_quad_130x96", "burgers2d_70")],
                         ids=lambda c: c[0])
def test_one_stage_mixed(case):
    name, P, u0, m0 = case
    print(f"[gpu] one-stage mixed {name}", flush=True)
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    ref = oracle_three_stages(P, u0, m0, dt, alpha)
    S = solver_for(P, precision="mixed")
    # the mixed path stores moments in FP32: feed it the rounded moments
    got = gpu_three_stages(S, P, u0, m0.astype(np.float32).astype(np.float64), dt, alpha,
                           inputs=ref[:2])
    for s in range(3):
        eu, em = state_err(P, got[s], ref[s])
        # averages: FP32 fluxes times dt/dx; moments: FP32 storage
        assert eu <= 2e-6 and em <= 2e-5, (name, s, eu, em)
    S.close()
