"""hwenou_step_noalloc (no device allocation, fixed device scratch) against
the existing entry point hwenou_stage (three stages through a handle) on the
same state, dt and alpha: equal bitwise (the same kernels; results do not
depend on the launch shape).  Two calls in a row, the second on a smaller
instance, so the second call must rebuild everything it reads from the
shared scratch array."""
import numpy as np
import pytest
import torch

import paper_2402_03074_amd as H
import workloads as W
from oracle.driver import Problem

from gpu_util import flat, solver_for, to_gpu

pytestmark = pytest.mark.gpu


def _case(kind, n):
    if kind == "euler2d":
        u, m = W.euler_2d_vortex_quadrant(n, seed=8100 + n, q=2)
        return Problem(2, "euler", (n, n), (0, 10, 0, 10)), u, m
    if kind == "burgers2d":
        u, m = W.burgers_2d_initial(n)
        return Problem(2, "burgers", (n, n), (0, 4, 0, 4)), u, m
    if kind == "euler1d":
        u, m = W.euler_1d_shocktube(n, seed=8300 + n)
        return Problem(1, "euler", n, (0, 1), bc="transmissive"), u, m
    u, m = W.advection_sine_1d(n)
    return Problem(1, "advection", n, (0, 2), adv=(1.0,)), u, m


def _by_stages(P, precision, u, m, dt, alpha):
    S = solver_for(P, precision=precision)
    uf, mf = flat(P, u, m)
    ug, mg = to_gpu(uf), to_gpu(mf, S.mom_dtype)
    dtg = torch.tensor([dt], dtype=torch.float64, device="cuda")
    al = torch.tensor([[alpha[0], alpha[1] if len(alpha) > 1 else 0.0]], dtype=torch.float64,
                      device="cuda")
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    u3, m3 = S.empty_state()
    S.stage(0, dtg, al, ug, mg, u1, m1)
    S.stage(1, dtg, al, u1, m1, u2, m2)
    S.stage(2, dtg, al, u2, m2, u3, m3)
    torch.cuda.synchronize()
    out = u3.cpu().numpy(), m3.cpu().numpy()
    S.close()
    return out


def _no_alloc(P, precision, u, m, dt, alpha, status):
    S = solver_for(P, precision=precision)  # only for its description and instance
    desc, inst = S.desc, S.instances[0]
    mom_dtype = S.mom_dtype
    S.close()
    uf, mf = flat(P, u, m)
    ug, mg = to_gpu(uf), to_gpu(mf, mom_dtype)
    dtg = torch.tensor([dt], dtype=torch.float64, device="cuda")
    al = torch.tensor([alpha[0], alpha[1] if len(alpha) > 1 else 0.0], dtype=torch.float64,
                      device="cuda")
    H.hwenou_step_noalloc(desc, inst, dtg, al, ug, mg, status)
    torch.cuda.synchronize()
    return ug.cpu().numpy(), mg.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,sizes", [("euler2d", (150, 70)), ("burgers2d", (96, 40)),
                                        ("euler1d", (9000, 3000)), ("advection1d", (800, 200))])
def test_no_alloc_step_equals_three_stages(kind, sizes, precision):
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n in sizes:  # two calls in a row, the second smaller
        print(f"[gpu] no-alloc step {kind} n={n} {precision}", flush=True)
        P, u, m = _case(kind, n)
        alpha = P.max_wavespeed(u)
        dt = P.dt_from(alpha, 0.6)
        ref = _by_stages(P, precision, u, m, dt, alpha)
        got = _no_alloc(P, precision, u, m, dt, alpha, status)
        assert np.array_equal(got[0], ref[0]), (kind, n, "averages")
        assert np.array_equal(got[1], ref[1]), (kind, n, "moments")
    assert int(status.item()) == 0


def test_no_alloc_step_rejects_an_instance_beyond_its_scratch():
    n = 600  # 2D Euler FP64 needs ~256 B per cell: 600^2 cells exceed 64 MiB
    P = Problem(2, "euler", (n, n), (0, 1, 0, 1))
    S = solver_for(P)
    desc, inst = S.desc, S.instances[0]
    S.close()
    u = torch.ones((4, n * n), dtype=torch.float64, device="cuda")
    m = torch.zeros((2, 4, n * n), dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    al = torch.ones(2, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HwenouError) as e:
        H.hwenou_step_noalloc(desc, inst, dt, al, u, m)
    assert e.value.code == H.HWENOU_ESCRATCH
