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

from gpu_util import (assert_mixed_stage_close, gpu_three_stages, oracle_three_stages,
                      solver_for, state_err, to_gpu, flat, unflat, rel_err)

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
    u, m = W.euler_2d_vortex_quadrant(130, 70, seed=3004, q=2)
    out.append(("euler2d_quad_130x70_single",
                Problem(2, "euler", (130, 70), (0, 10, 0, 10), char_decomp=2), u, m))
    u, m = W.euler_2d_vortex_quadrant(130, 70, seed=3005, q=2)
    out.append(("euler2d_quad_130x70_interface",
                Problem(2, "euler", (130, 70), (0, 10, 0, 10), char_decomp=3), u, m))
    u, m = W.euler_2d_vortex_quadrant(67, 40, seed=3006, q=2)
    out.append(("euler2d_quad_67x40_walls_interface",
                Problem(2, "euler", (67, 40), (0, 10, 0, 10), char_decomp=3,
                        bc=("reflective", "transmissive", "reflective", "transmissive")), u, m))
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


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
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


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
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
    assert_mixed_stage_close(name, P, u0, dt, alpha, got, ref)
    S.close()


# ---------------------------------------------------------------------------
# full workload sizes
# ---------------------------------------------------------------------------

def test_full_size_2d_euler_sampled_cells():
    """The 2048^2 benchmark workload, in the launch shape bench.py times: one
    stage on the GPU; 48 sampled cells recomputed by the oracle on 7x7 periodic
    patches (a cell's stage output depends on its 5x5 neighbourhood only)."""
    import torch
    import paper_2402_03074_amd as H
    n = 2048
    print("[gpu] full-size 2D sampled parity", flush=True)
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=3000, q=3)
    P = Problem(2, "euler", (n, n), (0.0, 10.0, 0.0, 10.0))
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    for precision in ("fp64", "mixed"):
        S = H.Solver(2, "euler", [H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0))],
                     precision=precision)
        ug = torch.tensor(u0.reshape(4, -1), device="cuda")
        mg = torch.tensor(m0.reshape(2, 4, -1), device="cuda").to(S.mom_dtype)
        al = torch.tensor([[alpha[0], alpha[1]]], dtype=torch.float64, device="cuda")
        dtg = torch.tensor([dt], dtype=torch.float64, device="cuda")
        uo, mo = S.empty_state()
        S.stage(0, dtg, al, ug, mg, uo, mo)
        torch.cuda.synchronize()
        got_u = uo.cpu().numpy().reshape(4, n, n)
        got_m = mo.double().cpu().numpy().reshape(2, 4, n, n)
        S.close()
        rng = np.random.default_rng(77)
        pts = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(44, 2))]
        pts += [(0, 0), (n - 1, n - 1), (0, n - 1), (1023, 1024)]
        m_in = m0 if precision == "fp64" else m0.astype(np.float32).astype(np.float64)
        Pp = Problem(2, "euler", (7, 7), (0.0, 7 * 10.0 / n, 0.0, 7 * 10.0 / n))
        tol_u, tol_m = (TOL_STAGE, TOL_STAGE) if precision == "fp64" else (2e-6, 2e-5)
        for (j, i) in pts:
            rows = [(j + d) % n for d in range(-3, 4)]
            cols = [(i + d) % n for d in range(-3, 4)]
            pu = u0[:, rows][:, :, cols]
            pm = m_in[:, :, rows][:, :, :, cols]
            ou, om, _ = Pp.stage(0, dt, alpha, pu, pm)
            for k in range(4):
                ref = ou[k, 3, 3]
                assert abs(got_u[k, j, i] - ref) <= tol_u * np.abs(u0[k]).max(), (precision, j, i, k)
                for d in range(2):
                    refm = om[d, k, 3, 3]
                    bound = tol_m * np.abs(m0[d, k]).max()
                    if precision == "mixed":
                        # on this fine grid the moments (~dx |grad u|) are small next to
                        # the FP32 rounding of the fluxes, which enters as dt/dx |u|
                        bound = max(bound, 1e-6 * dt / (10.0 / n) * np.abs(u0[k]).max())
                    assert abs(got_m[d, k, j, i] - refm) <= bound, (precision, j, i, k, d)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_1d_euler_all_cells(precision):
    """The 65 536-cell 1D Euler shock-tube workload, every cell, against the
    oracle after one step and after 100 steps.

    With 16 shocks and contacts the discrete dynamics amplify rounding: an
    oracle run whose input is perturbed by 1e-16 (relative) differs from the
    clean run by ~3e-9 (averages) and ~2e-8 (moments) after 100 steps.  No two
    implementations that round differently can agree better than that, so
    after 100 steps the bar is max(1e-10, 10 x that self-sensitivity),
    measured here on the same data."""
    import torch
    import paper_2402_03074_amd as H
    n = 65536
    print(f"[gpu] full-size 1D parity {precision}", flush=True)
    u0, m0 = W.euler_1d_shocktube(n, seed=2000)
    P = Problem(1, "euler", n, (0.0, 1.0), bc="transmissive")
    m_in = m0 if precision == "fp64" else m0.astype(np.float32).astype(np.float64)
    for steps in (1, 100):
        uo, mo, t, _ = P.advance(u0, m_in, cfl=0.6, max_steps=steps)
        S = solver_for(P, precision=precision)
        ug, mg = to_gpu(u0), to_gpu(m_in, S.mom_dtype)
        tg, sg = S.advance(ug, mg, 0.6, 1e30, steps)
        eu, em = state_err(P, (ug.cpu().numpy(), mg.double().cpu().numpy()), (uo, mo))
        S.close()
        if precision == "mixed":
            got = ug.cpu().numpy()
            l1 = max(np.abs(got[k] - uo[k]).mean() / np.abs(uo[k]).mean() for k in range(3))
            print(f"[gpu] mixed {steps} steps: rel Linf {eu:.2e} {em:.2e}, rel L1 {l1:.2e}",
                  flush=True)
            if steps == 1:
                assert eu <= 2e-6 and em <= 2e-5, (steps, eu, em)
            else:
                # FP32 rounding is amplified near the shocks like any perturbation
                # (see above); the L1 difference stays small
                assert l1 <= 1e-4, (steps, eu, em, l1)
            continue
        if steps == 1:
            # a whole step (three stages) within the one-stage bar: measured
            # 8e-16 / 4e-15
            assert eu <= TOL_STAGE and em <= TOL_STAGE, (eu, em)
            continue
        rng = np.random.default_rng(1)
        up = u0 * (1 + 1e-16 * rng.standard_normal(u0.shape))
        mp = m0 * (1 + 1e-16 * rng.standard_normal(m0.shape))
        ua, ma, _, _ = P.advance(up, mp, cfl=0.6, max_steps=steps)
        su, sm = state_err(P, (ua, ma), (uo, mo))
        print(f"[gpu] 100 steps: gpu {eu:.2e} {em:.2e}; oracle self-sensitivity "
              f"{su:.2e} {sm:.2e}", flush=True)
        assert eu <= max(TOL_STEPS, 10 * su) and em <= max(TOL_STEPS, 10 * sm), (eu, em, su, sm)


def test_full_batch_1d_sampled_instances():
    """The 512-instance 1D batch in one handle: three instances compared with
    the oracle after one step, averages and moments, within the one-stage bar
    (measured 8e-16 / 4e-15)."""
    import torch
    import paper_2402_03074_amd as H
    print("[gpu] full 1D batch sampled parity", flush=True)
    sizes, data = W.batch_1d_euler()
    insts, off = [], 0
    for nn in sizes:
        insts.append(H.make_inst(int(nn), 1, (0.0, 1.0), "transmissive", offset=off))
        off += int(nn)
    u = np.concatenate([d[0] for d in data], axis=1)
    m = np.concatenate([d[1] for d in data], axis=2)
    S = H.Solver(1, "euler", insts)
    ug, mg = to_gpu(u), to_gpu(m)
    S.advance(ug, mg, 0.6, 1e30, 1)
    got, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    for k in (0, 255, 511):
        a, b = insts[k].offset, insts[k].offset + insts[k].nx
        P = Problem(1, "euler", insts[k].nx, (0.0, 1.0), bc="transmissive")
        uo, mo, _, _ = P.advance(data[k][0], data[k][1], cfl=0.6, max_steps=1)
        eu, em = state_err(P, (got[:, a:b], got_m[:, :, a:b]), (uo, mo))
        assert eu <= TOL_STAGE and em <= TOL_STAGE, (k, eu, em)
    S.close()


def test_full_batch_2d_sampled_instances():
    """The 64-instance 2D batch (grids of 256^2 to 1024^2, 22 M cells) in one
    handle, at the default launch shape (results do not depend on it, see
    test_launch_shape_invariance): one step, then the smallest, a median and
    the largest instance compared whole with the oracle, within the one-stage
    bar (measured 1e-15 / 1e-14)."""
    import torch
    import paper_2402_03074_amd as H
    print("[gpu] full 2D batch sampled parity: generating", flush=True)
    sides, data = W.batch_2d_euler()
    insts, off = [], 0
    for side in sides:
        insts.append(H.make_inst(int(side), int(side), (0.0, 10.0, 0.0, 10.0), "periodic",
                                 offset=off))
        off += int(side) ** 2
    u = np.concatenate([d[0].reshape(4, -1) for d in data], axis=1)
    m = np.concatenate([d[1].reshape(2, 4, -1) for d in data], axis=2)
    S = H.Solver(2, "euler", insts)
    ug, mg = to_gpu(u), to_gpu(m)
    S.advance(ug, mg, 0.6, 1e30, 1)
    torch.cuda.synchronize()
    got_u, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    S.close()
    del ug, mg
    order = np.argsort(sides, kind="stable")
    for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        n = int(sides[k])
        print(f"[gpu] full 2D batch: instance {k} ({n}^2) against the oracle", flush=True)
        a, b = insts[k].offset, insts[k].offset + n * n
        P = Problem(2, "euler", (n, n), (0.0, 10.0, 0.0, 10.0))
        uo, mo, _, _ = P.advance(data[k][0], data[k][1], cfl=0.6, max_steps=1)
        got = (got_u[:, a:b].reshape(4, n, n), got_m[:, :, a:b].reshape(2, 4, n, n))
        eu, em = state_err(P, got, (uo, mo))
        assert eu <= TOL_STAGE and em <= TOL_STAGE, (k, n, eu, em)


@pytest.mark.parametrize("weights", ["zq", "linear"])
@pytest.mark.parametrize("dim", [1, 2])
def test_weight_modes_one_step(weights, dim):
    """The scale-dependent (ZQ) and linear weights run in kernels that take
    the mode at run time; the default scale-invariant weights are covered by
    every other parity test."""
    if dim == 1:
        u, m = W.euler_1d_shocktube(1000, seed=3101)
        P = Problem(1, "euler", 1000, (0, 1), bc="transmissive", weights=weights)
    else:
        u, m = W.euler_2d_vortex_quadrant(70, 64, seed=3100, q=2)
        P = Problem(2, "euler", (70, 64), (0, 10, 0, 10), weights=weights)
    alpha = P.max_wavespeed(u)
    dt = P.dt_from(alpha, 0.4)
    ref = oracle_three_stages(P, u, m, dt, alpha)
    S = solver_for(P)
    got = gpu_three_stages(S, P, u, m, dt, alpha, inputs=ref[:2])
    for s in range(3):
        eu, em = state_err(P, got[s], ref[s])
        assert eu <= TOL_STAGE and em <= TOL_STAGE, (weights, dim, s, eu, em)
    S.close()


def _degenerate_cases():
    """Grids at and around the kernels' tile edges: the smallest grid the
    method allows (3 cells a side, where the stencils of a periodic grid wrap
    onto themselves), one 62-column strip or 62-cell tile exactly, one more,
    and a grid of 64; each with periodic, outflow and wall sides."""
    out = []
    for nx, ny in ((3, 3), (3, 5), (62, 3), (63, 4), (64, 7)):
        u, m = W.euler_2d_vortex_quadrant(nx, ny, seed=5000 + nx + 100 * ny, q=2)
        for bc in ("periodic", "transmissive", "reflective"):
            out.append((f"2d_{nx}x{ny}_{bc}",
                        Problem(2, "euler", (nx, ny), (0, 10, 0, 10), bc=bc), u, m))
    for n in (3, 4, 61, 62, 63, 64, 125):
        u, m = W.random_smooth_1d(n, 3, seed=5100 + n, positive_euler=True)
        for bc in ("periodic", "transmissive", "reflective"):
            out.append((f"1d_{n}_{bc}", Problem(1, "euler", n, (0, 1), bc=bc), u, m))
    return out


DEGENERATE = _degenerate_cases()


@pytest.mark.parametrize("case", DEGENERATE, ids=[c[0] for c in DEGENERATE])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_degenerate_sizes_one_step(case, precision):
    """One Runge-Kutta step (the three stages) on the smallest and
    tile-edge grid sizes against the oracle, at the one-stage bar of each
    precision."""
    name, P, u, m = case
    print(f"[gpu] degenerate size {name} {precision}", flush=True)
    alpha = P.max_wavespeed(u)
    dt = P.dt_from(alpha, 0.5)
    if precision == "mixed":
        m = m.astype(np.float32).astype(np.float64)  # the moments it stores
    ref = oracle_three_stages(P, u, m, dt, alpha)
    S = solver_for(P, precision=precision)
    got = gpu_three_stages(S, P, u, m, dt, alpha, inputs=ref[:2])
    if precision == "mixed":
        assert_mixed_stage_close(name, P, u, dt, alpha, got, ref)
    else:
        for s in range(3):
            eu, em = state_err(P, got[s], ref[s], floor=1e-3)
            assert eu <= TOL_STAGE and em <= TOL_STAGE, (name, s, eu, em)
    S.close()


def test_full_size_2d_euler_full_step_sampled_cells():
    """The 2048^2 benchmark workload: one whole Runge-Kutta step (the three
    stage kernels) on the GPU, in the launch shape bench.py times; 24 sampled
    cells recomputed by the oracle on 15x15 periodic patches (after three
    stages a cell depends on its 13x13 neighbourhood, and the wrap of the
    patch reaches at most 6 cells in from its edge)."""
    import torch
    import paper_2402_03074_amd as H
    n, r = 2048, 7
    print("[gpu] full-size 2D full-step sampled parity", flush=True)
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=3000, q=3)
    P = Problem(2, "euler", (n, n), (0.0, 10.0, 0.0, 10.0))
    alpha = P.max_wavespeed(u0)
    dt = P.dt_from(alpha, 0.6)
    S = H.Solver(2, "euler", [H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0))])
    ug = torch.tensor(u0.reshape(4, -1), device="cuda")
    mg = torch.tensor(m0.reshape(2, 4, -1), device="cuda")
    al = torch.tensor([[alpha[0], alpha[1]]], dtype=torch.float64, device="cuda")
    dtg = torch.tensor([dt], dtype=torch.float64, device="cuda")
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    u3, m3 = S.empty_state()
    S.stage(0, dtg, al, ug, mg, u1, m1)
    S.stage(1, dtg, al, u1, m1, u2, m2)
    S.stage(2, dtg, al, u2, m2, u3, m3)
    torch.cuda.synchronize()
    got_u = u3.cpu().numpy().reshape(4, n, n)
    got_m = m3.cpu().numpy().reshape(2, 4, n, n)
    S.close()
    rng = np.random.default_rng(78)
    pts = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(22, 2))] + [(0, 0), (2047, 1)]
    h = 10.0 / n
    Pp = Problem(2, "euler", (2 * r + 1, 2 * r + 1), (0.0, (2 * r + 1) * h, 0.0, (2 * r + 1) * h))
    for (j, i) in pts:
        rows = [(j + d) % n for d in range(-r, r + 1)]
        cols = [(i + d) % n for d in range(-r, r + 1)]
        pu = np.ascontiguousarray(u0[:, rows][:, :, cols])
        pm = np.ascontiguousarray(m0[:, :, rows][:, :, :, cols])
        u_, m_, base = Pp.stage(0, dt, alpha, pu, pm)
        u_, m_, _ = Pp.stage(1, dt, alpha, u_, m_, base)
        u_, m_, _ = Pp.stage(2, dt, alpha, u_, m_, base)
        for k in range(4):
            scale = np.abs(u0[k]).max()
            assert abs(got_u[k, j, i] - u_[k, r, r]) <= TOL_STAGE * scale, (j, i, k)
            for d in range(2):
                mscale = np.abs(m0[d, k]).max()
                assert abs(got_m[d, k, j, i] - m_[d, k, r, r]) <= TOL_STAGE * mscale, (j, i, k, d)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_average_stencils(precision):
    """Stencils whose five-cell cross has zero averages (u_ave = 0: the
    nonlinear weights reduce to the linear ones, by the remark after
    Eq. (2.11)) on the GPU: averages non-zero only on a lattice of every third
    cell in x and y, so every cell at (1, 1) mod 3 has a zero cross and
    non-zero corners; random moments.  One step against the oracle."""
    n = 33
    rng = np.random.default_rng(91)
    u = np.zeros((1, n, n))
    u[0, ::3, ::3] = rng.uniform(0.5, 1.5, (11, 11)) * rng.choice([-1.0, 1.0], (11, 11))
    m = rng.uniform(-0.2, 0.2, (2, 1, n, n))
    P = Problem(2, "advection", (n, n), (0, 1, 0, 1), adv=(1.0, -0.5))
    alpha = P.max_wavespeed(u)
    dt = P.dt_from(alpha, 0.4)
    print(f"[gpu] zero-average stencils {precision}", flush=True)
    ref = oracle_three_stages(P, u, m, dt, alpha)
    S = solver_for(P, precision=precision)
    if precision == "fp64":
        got = gpu_three_stages(S, P, u, m, dt, alpha, inputs=ref[:2])
        for s in range(3):
            eu, em = state_err(P, got[s], ref[s])
            assert eu <= TOL_STAGE and em <= TOL_STAGE, (s, eu, em)
    else:
        got = gpu_three_stages(S, P, u, m.astype(np.float32).astype(np.float64), dt, alpha,
                               inputs=ref[:2])
        assert_mixed_stage_close("zero_average", P, u, dt, alpha, got, ref)
    S.close()
