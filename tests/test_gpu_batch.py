"""GPU tests of the batched persistent launch, graph replay, resumption,
launch-shape invariance, conservation and the non-physical-state report.

Bitwise comparisons hold because every cell is computed by the same code
path whatever the batch layout or launch shape, and the wave-speed
reductions are max-reductions (order independent)."""
import numpy as np
import pytest
import torch

import paper_2402_03074_amd as H
import workloads as W
from oracle.driver import Problem

from gpu_util import flat, rel_err, solver_for, to_gpu

pytestmark = pytest.mark.gpu


def _batch_1d(sizes, seed):
    insts, us, ms, off = [], [], [], 0
    for k, n in enumerate(sizes):
        u, m = W.euler_1d_shocktube(int(n), seed + k)
        insts.append(H.make_inst(n, 1, (0.0, 1.0), "transmissive", offset=off))
        us.append(u)
        ms.append(m)
        off += int(n)
    return insts, np.concatenate(us, axis=1), np.concatenate(ms, axis=2)


def _batch_2d(sides, seed, precision="fp64"):
    insts, us, ms, off = [], [], [], 0
    for k, n in enumerate(sides):
        u, m = W.euler_2d_vortex_quadrant(int(n), seed=seed + k, q=2)
        insts.append(H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0), "periodic", offset=off))
        us.append(u.reshape(4, -1))
        ms.append(m.reshape(2, 4, -1))
        off += int(n) * int(n)
    return insts, np.concatenate(us, axis=1), np.concatenate(ms, axis=2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_1d_equals_single_instances(precision):
    print(f"[gpu] batched 1D {precision}", flush=True)
    sizes = W.log_uniform_sizes(24, 64, 3000, seed=4100)
    insts, u, m = _batch_1d(sizes, 4101)
    S = H.Solver(1, "euler", insts, precision=precision)
    ug, mg = to_gpu(u), to_gpu(m, S.mom_dtype)
    t, steps = S.advance(ug, mg, 0.6, 0.05, 40)
    got_u, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    S.close()
    for k, I in enumerate(insts):
        a, b = I.offset, I.offset + I.nx
        S1 = H.Solver(1, "euler", [H.make_inst(I.nx, 1, (0.0, 1.0), "transmissive")],
                      precision=precision)
        u1, m1 = to_gpu(u[:, a:b]), to_gpu(m[:, :, a:b], S1.mom_dtype)
        t1, s1 = S1.advance(u1, m1, 0.6, 0.05, 40)
        assert t1[0] == t[k] and s1[0] == steps[k]
        assert np.array_equal(u1.cpu().numpy(), got_u[:, a:b])
        assert np.array_equal(m1.cpu().numpy(), got_m[:, :, a:b])
        S1.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_2d_equals_single_instances(precision):
    print(f"[gpu] batched 2D {precision}", flush=True)
    sides = [70, 64, 131, 33, 96]
    insts, u, m = _batch_2d(sides, 5100)
    S = H.Solver(2, "euler", insts, precision=precision)
    ug, mg = to_gpu(u), to_gpu(m, S.mom_dtype)
    t, steps = S.advance(ug, mg, 0.6, 1e30, 6)
    got_u, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    S.close()
    for k, I in enumerate(insts):
        a, b = I.offset, I.offset + I.nx * I.ny
        S1 = H.Solver(2, "euler", [H.make_inst(I.nx, I.ny, (0.0, 10.0, 0.0, 10.0))],
                      precision=precision)
        u1, m1 = to_gpu(u[:, a:b]), to_gpu(m[:, :, a:b], S1.mom_dtype)
        t1, s1 = S1.advance(u1, m1, 0.6, 1e30, 6)
        assert t1[0] == t[k] and s1[0] == steps[k] == 6
        assert np.array_equal(u1.cpu().numpy(), got_u[:, a:b])
        assert np.array_equal(m1.cpu().numpy(), got_m[:, :, a:b])
        S1.close()


@pytest.mark.parametrize("char_decomp", [1, 2])
def test_batched_2d_mixed_boundaries_equals_single_instances(char_decomp):
    """One handle holding instances with different boundary sides (walls,
    outflow, periodic) gives, bitwise, the single-instance results, for the
    split and the single-projection reconstruction."""
    print(f"[gpu] batched 2D, mixed boundaries, char_decomp {char_decomp}", flush=True)
    sides = [70, 40, 96, 33]
    bcs = [("reflective",) * 4,
           ("reflective", "transmissive", "periodic", "periodic"),
           ("periodic", "periodic", "transmissive", "reflective"),
           ("transmissive",) * 4]
    insts, us, ms, off = [], [], [], 0
    for k, (n, bc) in enumerate(zip(sides, bcs)):
        u1, m1 = W.euler_2d_vortex_quadrant(n, seed=5300 + k, q=2)
        insts.append(H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0), bc, offset=off))
        us.append(u1.reshape(4, -1))
        ms.append(m1.reshape(2, 4, -1))
        off += n * n
    u, m = np.concatenate(us, axis=1), np.concatenate(ms, axis=2)
    S = H.Solver(2, "euler", insts, char_decomp=char_decomp)
    ug, mg = to_gpu(u), to_gpu(m)
    t, steps = S.advance(ug, mg, 0.6, 1e30, 5)
    got_u, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    S.close()
    for k, (I, bc) in enumerate(zip(insts, bcs)):
        a, b = I.offset, I.offset + I.nx * I.ny
        S1 = H.Solver(2, "euler", [H.make_inst(I.nx, I.ny, (0.0, 10.0, 0.0, 10.0), bc)],
                      char_decomp=char_decomp)
        u1, m1 = to_gpu(u[:, a:b]), to_gpu(m[:, :, a:b])
        t1, s1 = S1.advance(u1, m1, 0.6, 1e30, 5)
        assert t1[0] == t[k] and s1[0] == steps[k] == 5
        assert np.array_equal(u1.cpu().numpy(), got_u[:, a:b]), k
        assert np.array_equal(m1.cpu().numpy(), got_m[:, :, a:b]), k
        S1.close()


def test_batched_1d_walls_equals_single_instances():
    """1D: a batch of blast-wave-like instances between walls next to outflow
    instances equals the single-instance runs bitwise."""
    print("[gpu] batched 1D walls", flush=True)
    sizes = [300, 77, 1000, 64]
    bcs = ["reflective", "transmissive", ("reflective", "transmissive"), "reflective"]
    insts, us, ms, off = [], [], [], 0
    for k, (n, bc) in enumerate(zip(sizes, bcs)):
        u1, m1 = W.euler_1d_shocktube(n, 5400 + k)
        insts.append(H.make_inst(n, 1, (0.0, 1.0), bc, offset=off))
        us.append(u1)
        ms.append(m1)
        off += n
    u, m = np.concatenate(us, axis=1), np.concatenate(ms, axis=2)
    S = H.Solver(1, "euler", insts)
    ug, mg = to_gpu(u), to_gpu(m)
    t, steps = S.advance(ug, mg, 0.6, 0.02, 10 ** 5)
    got_u, got_m = ug.cpu().numpy(), mg.cpu().numpy()
    S.close()
    for k, (I, bc) in enumerate(zip(insts, bcs)):
        a, b = I.offset, I.offset + I.nx
        S1 = H.Solver(1, "euler", [H.make_inst(I.nx, 1, (0.0, 1.0), bc)])
        u1, m1 = to_gpu(u[:, a:b]), to_gpu(m[:, :, a:b])
        t1, s1 = S1.advance(u1, m1, 0.6, 0.02, 10 ** 5)
        assert t1[0] == t[k] and s1[0] == steps[k]
        assert np.array_equal(u1.cpu().numpy(), got_u[:, a:b]), k
        assert np.array_equal(m1.cpu().numpy(), got_m[:, :, a:b]), k
        S1.close()


def test_batch_instances_finish_at_their_own_final_time():
    """Instances of different sizes take different time steps; each stops at
    t_final exactly, matching the oracle run of that instance."""
    sizes = [50, 200, 90]
    insts, u, m = _batch_1d(sizes, 4200)
    S = H.Solver(1, "euler", insts)
    ug, mg = to_gpu(u), to_gpu(m)
    t, steps = S.advance(ug, mg, 0.6, 0.03, 10 ** 6)
    for k, I in enumerate(insts):
        a, b = I.offset, I.offset + I.nx
        P = Problem(1, "euler", I.nx, (0.0, 1.0), bc="transmissive")
        uo, mo, to, so = P.advance(u[:, a:b], m[:, :, a:b], cfl=0.6, t_final=0.03)
        assert abs(t[k] - 0.03) < 1e-15 and steps[k] == so
        eu = rel_err(ug.cpu().numpy()[:, a:b], uo, 1)
        assert eu < 1e-11, (k, eu)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,big", [(1, False), (2, False), (1, True), (2, True)])
def test_graph_replay_equals_eager_stages(dim, big, precision):
    """Graph replays take each step's alpha from the wave speeds that the
    stage-2 kernel reduces while it writes the step's result; the eager
    stages here take it from the separate max-wave-speed kernel.  Equal
    states after 5 steps pin the fused reduction bitwise.  The small grids
    reduce into one accumulator per instance; the big ones (about 1000 waves
    on the one instance) into several, whose maximum the finish kernel takes."""
    print(f"[gpu] graph vs eager dim={dim} big={big} {precision}", flush=True)
    if dim == 1:
        n = 65536 if big else 3000
        u0, m0 = W.euler_1d_shocktube(n, seed=5201)
        P = Problem(1, "euler", n, (0, 1), bc="transmissive")
        dx = 1.0 / n
    else:
        n = 512 if big else 96
        u0, m0 = W.euler_2d_vortex_quadrant(n, seed=5200, q=2)
        P = Problem(2, "euler", (n, n), (0, 10, 0, 10))
        dx = 10.0 / n
    uf, mf = flat(P, u0, m0)
    S = solver_for(P, precision=precision)
    mdt = S.mom_dtype
    ua, ma = to_gpu(uf), to_gpu(mf, mdt)
    S.advance(ua, ma, 0.6, 1e30, 5)
    ub, mb = to_gpu(uf), to_gpu(mf, mdt)
    for _ in range(5):
        alpha = S.max_wavespeed(ub)
        a = alpha.cpu().numpy()[0]
        # the device's time step, in its order of operations
        step = 0.6 * dx / a[0] if dim == 1 else 0.6 / (a[0] / dx + a[1] / dx)
        dt = torch.tensor([step], dtype=torch.float64, device="cuda")
        u1, m1 = S.empty_state()
        u2, m2 = S.empty_state()
        S.stage(0, dt, alpha, ub, mb, u1, m1)
        S.stage(1, dt, alpha, u1, m1, u2, m2)
        S.stage(2, dt, alpha, u2, m2, ub, mb)  # in place into the base, as advance does
    torch.cuda.synchronize()
    assert torch.equal(ua, ub) and torch.equal(ma, mb)
    S.close()


def test_resume_is_bitwise():
    n = 80
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=5300, q=2)
    P = Problem(2, "euler", (n, n), (0, 10, 0, 10))
    uf, mf = flat(P, u0, m0)
    S = solver_for(P, precision="mixed")
    ua, ma = to_gpu(uf), to_gpu(mf, torch.float32)
    S.advance(ua, ma, 0.6, 1e30, 8)
    ub, mb = to_gpu(uf), to_gpu(mf, torch.float32)
    S.advance(ub, mb, 0.6, 1e30, 4)
    S.advance(ub, mb, 0.6, 1e30, 4)
    assert torch.equal(ua, ub) and torch.equal(ma, mb)
    S.close()


@pytest.mark.parametrize("dim", [1, 2])
def test_launch_shape_invariance(dim):
    """Different persistent-launch shapes give bitwise identical results."""
    if dim == 1:
        u0, m0 = W.euler_1d_shocktube(5000, seed=5400)
        P = Problem(1, "euler", 5000, (0, 1), bc="transmissive")
    else:
        u0, m0 = W.euler_2d_vortex_quadrant(150, 90, seed=5401, q=2)
        P = Problem(2, "euler", (150, 90), (0, 10, 0, 10))
    uf, mf = flat(P, u0, m0)
    outs = []
    for wpc, rows in ((1, 0), (4, 7), (16, 0), (3, 33)):
        S = solver_for(P)
        S.set_launch(wpc, rows)
        ug, mg = to_gpu(uf), to_gpu(mf)
        S.advance(ug, mg, 0.6, 1e30, 3)
        outs.append((ug.cpu().numpy(), mg.cpu().numpy()))
        S.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_conservation_2d_euler(precision):
    n = 128
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=5500, q=2)
    P = Problem(2, "euler", (n, n), (0, 10, 0, 10))
    uf, mf = flat(P, u0, m0)
    S = solver_for(P, precision=precision)
    ug, mg = to_gpu(uf), to_gpu(mf, S.mom_dtype)
    S.advance(ug, mg, 0.6, 1e30, 100)
    u1 = ug.cpu().numpy()
    # extended-precision sums; a conservation error in the flux bookkeeping
    # would show at the level of the fluxes (1e-3 and above), round-off of
    # 300 stages of shock data stays within a few hundred ulp of the total
    total = np.abs(uf).sum(axis=1)
    drift = np.abs(np.array([np.sum(x.astype(np.longdouble)) for x in u1])
                   - np.array([np.sum(x.astype(np.longdouble)) for x in uf]))
    assert np.all(drift <= 1e-13 * total), drift / total
    S.close()


def test_nonphysical_state_is_reported():
    n = 40
    u0, m0 = W.euler_2d_vortex_quadrant(n, seed=5600, q=2)
    u0 = u0.copy()
    u0[3, 7, 11] = -1.0  # negative energy: negative pressure in one cell
    P = Problem(2, "euler", (n, n), (0, 10, 0, 10))
    uf, mf = flat(P, u0, m0)
    S = solver_for(P)
    ug, mg = to_gpu(uf), to_gpu(mf)
    with pytest.raises(H.NonPhysicalState):
        S.advance(ug, mg, 0.6, 1e30, 3)
    S.close()


def test_stage_api_rejects_stage1_before_stage0():
    n = 16
    P = Problem(2, "euler", (n, n), (0, 1, 0, 1))
    S = solver_for(P)
    u, m = S.empty_state()
    u2, m2 = S.empty_state()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    al = torch.ones((1, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HwenouError) as e:
        S.stage(1, dt, al, u, m, u2, m2)
    assert e.value.code == H.HWENOU_EINVAL
    with pytest.raises(H.HwenouError):
        S.stage(0, dt, al, u, m, u, m)  # aliasing in and out
    # hwenou_advance runs its own stage 0 (replacing the stored v^n) and
    # clears the record: a stage 1 after it needs a new stage 0
    u.copy_(torch.tensor([1.0, 0.2, 0.1, 2.5], dtype=torch.float64,
                         device="cuda")[:, None].expand_as(u))
    m.zero_()
    S.stage(0, dt, al, u, m, u2, m2)
    S.advance(u, m, 0.6, 1e30, 1)
    with pytest.raises(H.HwenouError) as e:
        S.stage(1, dt, al, u2, m2, u, m)
    assert e.value.code == H.HWENOU_EINVAL
    S.close()


def test_autotuner_keeps_results_bitwise(tmp_path, monkeypatch):
    monkeypatch.setenv("HWENOU_TUNE_CACHE", str(tmp_path / "tune.json"))
    sides = [100, 64, 37]
    insts, u, m = _batch_2d(sides, 5700)
    ref = H.Solver(2, "euler", insts, precision="mixed")
    ur, mr = to_gpu(u), to_gpu(m, torch.float32)
    ref.advance(ur, mr, 0.6, 1e30, 3)
    S = H.Solver(2, "euler", insts, precision="mixed")
    ug, mg = to_gpu(u), to_gpu(m, torch.float32)
    w, r = S.autotune(ug, mg, reps=2)
    assert 1 <= w <= 32 and r >= 0
    assert (tmp_path / "tune.json").exists()
    S.advance(ug, mg, 0.6, 1e30, 3)
    assert torch.equal(ug, ur) and torch.equal(mg, mr)
    # a second handle of the same class takes the cached shape
    S2 = H.Solver(2, "euler", insts, precision="mixed")
    assert S2.autotune(ug, mg) == (w, r)
    for s_ in (ref, S, S2):
        s_.close()


def test_zero_wave_speed_reaches_final_time():
    """Advection at zero velocity: every flux vanishes and the CFL bound is
    infinite, so one step covers the whole interval; the averages are
    unchanged up to the rounding of the Runge-Kutta combinations."""
    print("[gpu] zero wave speed", flush=True)
    P = Problem(1, "advection", 64, (0, 2), adv=(0.0,))
    u0, m0 = W.advection_sine_1d(64)
    S = solver_for(P)
    ug, mg = to_gpu(u0), to_gpu(m0)
    t, st = S.advance(ug, mg, 0.6, 1.5, 100)
    assert t == [1.5] and st == [1]
    assert np.abs(ug.cpu().numpy() - u0).max() <= 1e-15 * np.abs(u0).max()
    S.close()


def test_non_finite_state_is_reported():
    """A NaN in the averages stops the instance with ENONPHYSICAL."""
    P = Problem(1, "euler", 64, (0, 1), bc="transmissive")
    u0, m0 = W.euler_1d_shocktube(64, seed=77)
    u0[0, 10] = np.nan
    S = solver_for(P)
    ug, mg = to_gpu(u0), to_gpu(m0)
    with pytest.raises(H.NonPhysicalState) as e:
        S.advance(ug, mg, 0.6, 1e30, 3)
    assert e.value.steps == [0] and e.value.t == [0.0] and e.value.flags == [1]
    S.close()


def _vacuum_1d(n):
    """Two streams leaving each other at Mach ~10: a vacuum forms and the
    scheme (which has no positivity limiter) leaves the physical states
    within a few steps (the oracle fails in its third step)."""
    x = (np.arange(n) + 0.5) / n
    rho = np.ones(n)
    u = np.where(x < 0.5, -6.0, 6.0)
    p = 0.2 * np.ones(n)
    U = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
    return U, np.zeros((1, 3, n))


@pytest.mark.parametrize("bad", ["nan", "vacuum"])
def test_failed_instance_stops_alone(bad):
    """Per-instance failure: the instance whose state leaves the physical
    states stops after the step in which that happened (its t and step count
    say where, its flag is set), while the other instances run every step
    and equal runs of themselves alone, bitwise."""
    print(f"[gpu] failed instance stops alone: {bad}", flush=True)
    sizes = [64, 80, 48]
    insts, u, m = _batch_1d(sizes, 7700)
    if bad == "nan":
        u[0, 64 + 10] = np.nan  # instance 1, before the first step
    else:
        uv, mv = _vacuum_1d(80)
        u[:, 64:144] = uv
        m[:, :, 64:144] = mv
    S = H.Solver(1, "euler", insts)
    ug, mg = to_gpu(u), to_gpu(m)
    steps = 12
    with pytest.raises(H.NonPhysicalState) as e:
        S.advance(ug, mg, 0.6, 1e30, steps)
    st, t, flags = e.value.steps, e.value.t, e.value.flags
    assert flags == [0, 1, 0], flags
    assert st[0] == st[2] == steps
    if bad == "nan":
        assert st[1] == 0 and t[1] == 0.0
    else:
        assert 1 <= st[1] < steps and 0.0 < t[1] < t[0], (st, t)
    assert H.hwenou_inst_status(S.h) == [0, 0, 0]  # read and cleared
    out = ug.cpu().numpy()
    S.close()
    for k, off in ((0, 0), (2, 144)):
        n = sizes[k]
        S1 = H.Solver(1, "euler", [H.make_inst(n, 1, (0.0, 1.0), "transmissive")])
        u1, m1 = to_gpu(np.ascontiguousarray(u[:, off:off + n])), \
            to_gpu(np.ascontiguousarray(m[:, :, off:off + n]))
        S1.advance(u1, m1, 0.6, 1e30, steps)
        assert np.array_equal(u1.cpu().numpy(), out[:, off:off + n]), k
        S1.close()
