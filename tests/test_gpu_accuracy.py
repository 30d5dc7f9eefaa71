"""Accuracy of the GPU path against exact solutions: the fifth-order rate of
both precisions on the smooth Euler problems of Section 3.1, and equal L1
error of the mixed and FP64 forms where the discretisation error is well
above the FP32 floor."""
import math
import os

import numpy as np
import pytest
import torch

import paper_2402_03074_amd as H
import workloads as W

pytestmark = pytest.mark.gpu


def _run_1d_euler(n, precision):
    u0, m0 = W.euler_1d_sine(n)
    ue, _ = W.euler_1d_sine(n, t=2.0)
    S = H.Solver(1, "euler", [H.make_inst(n, 1, (0.0, 2.0))], precision=precision)
    ug = torch.tensor(u0, device="cuda")
    mg = torch.tensor(m0, device="cuda").to(S.mom_dtype)
    # dt ~ dx^(5/3): advance in chunks with a fixed step computed here
    dx = 2.0 / n
    alpha = 1.0 + np.sqrt(1.4 * 1.0 / 0.8)  # bound of |u| + c for rho >= 0.8
    dt = 0.6 * dx ** (5.0 / 3.0) / alpha
    steps = int(np.ceil(2.0 / dt))
    dt = 2.0 / steps
    dtg = torch.tensor([dt], dtype=torch.float64, device="cuda")
    al = S.max_wavespeed(ug)
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    for _ in range(steps):
        al = S.max_wavespeed(ug)
        S.stage(0, dtg, al, ug, mg, u1, m1)
        S.stage(1, dtg, al, u1, m1, u2, m2)
        S.stage(2, dtg, al, u2, m2, ug, mg)
    torch.cuda.synchronize()
    S.close()
    return np.abs(ug.cpu().numpy()[0] - ue[0]).mean()


def test_1d_euler_fifth_order_both_precisions():
    print("[gpu] 1D Euler accuracy", flush=True)
    e = {(p, n): _run_1d_euler(n, p) for p in ("fp64", "mixed") for n in (20, 40, 80)}
    print({k: f"{v:.3e}" for k, v in e.items()}, flush=True)
    for p in ("fp64", "mixed"):
        assert np.log2(e[(p, 20)] / e[(p, 40)]) > 4.5
    assert np.log2(e[("fp64", 40)] / e[("fp64", 80)]) > 4.5
    # the mixed form adds at most an FP32 floor of 1e-7 (measured ~1e-7 after
    # ~3700 steps at N = 80) to the discretisation error, and matches FP64 to
    # 1% where the error is far above that floor
    floor = 1.0e-7
    for n in (20, 40, 80):
        assert e[("mixed", n)] <= e[("fp64", n)] + floor
    assert abs(e[("mixed", 20)] - e[("fp64", 20)]) <= 0.01 * e[("fp64", 20)]


def _vortex_l1(n, T, precision, char_decomp=True):
    u0, m0 = W.euler_2d_vortex(n)
    ue, _ = W.euler_2d_vortex(n, t=T)
    S = H.Solver(2, "euler", [H.make_inst(n, n, (0.0, 10.0, 0.0, 10.0))], precision=precision,
                 char_decomp=char_decomp)
    ug = torch.tensor(u0.reshape(4, -1), device="cuda")
    mg = torch.tensor(m0.reshape(2, 4, -1), device="cuda").to(S.mom_dtype)
    t, s = S.advance(ug, mg, 0.6, T, 10 ** 6)
    assert abs(t[0] - T) < 1e-14
    err = np.abs(ug.cpu().numpy()[0].reshape(n, n) - ue[0]).mean()
    S.close()
    return err


def test_2d_vortex_mixed_matches_fp64_l1_error():
    """Smooth isentropic vortex (strength 5) translated by a uniform flow:
    the L1 density error of the mixed form equals FP64's within 1% where the
    discretisation error is far above the FP32 floor (64^2), and exceeds it
    by no more than that floor (measured ~1e-7 after ~100 steps) at 128^2."""
    print("[gpu] 2D vortex accuracy", flush=True)
    e = {(p, n): _vortex_l1(n, 1.0, p) for p in ("fp64", "mixed") for n in (64, 128)}
    print({k: f"{v:.4e}" for k, v in e.items()}, flush=True)
    assert abs(e[("mixed", 64)] - e[("fp64", 64)]) <= 0.01 * e[("fp64", 64)]
    assert e[("mixed", 128)] <= e[("fp64", 128)] + 1.5e-7
    assert e[("fp64", 64)] / e[("fp64", 128)] > 8.0  # at least third order in time


def test_2d_vortex_projection_modes():
    """Cost/accuracy of the reconstruction variables on the smooth vortex
    (FP64): the single x-projection, the component-wise reconstruction and
    the per-interface bases keep the error of the direction-split
    characteristic scheme within a factor 1.5 and converge at least at third
    order (the time error) between 64^2 and 128^2."""
    print("[gpu] 2D vortex, projection modes", flush=True)
    e = {(c, n): _vortex_l1(n, 1.0, "fp64", c) for c in (1, 2, 0, 3) for n in (64, 128)}
    print({k: f"{v:.4e}" for k, v in e.items()}, flush=True)
    for c in (2, 0, 3):
        for n in (64, 128):
            assert e[(c, n)] <= 1.5 * e[(1, n)]
        assert e[(c, 64)] / e[(c, 128)] > 8.0


def _table(example):
    path = os.path.join(os.path.dirname(__file__), "golden", "accuracy_tables.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            r = line.split()
            if r and not r[0].startswith("#") and r[0] == example:
                out[int(r[1])] = (float(r[2]), float(r[3]))
    return out


def _run_2d_table(eq, n, L, T, alpha_bound):
    """FP64 run to T with dt = CFL / (a/dx^(5/3) + a/dy^(5/3)), CFL 0.6, a the
    wave-speed bound of the data, and the Lax-Friedrichs alpha of every step
    from the cell averages; returns (L-inf, L1) of the density/u error."""
    if eq == "euler":
        u0, m0 = W.euler_2d_sine(n, L=L)
        ue, _ = W.euler_2d_sine(n, t=T, L=L)
    else:
        u0, m0 = W.burgers_2d_initial(n)
        ue, _ = W.burgers_2d_exact_moments(n, T)
    S = H.Solver(2, eq, [H.make_inst(n, n, (0.0, L, 0.0, L))])
    dx = L / n
    dt = 0.6 / (2.0 * alpha_bound / dx ** (5.0 / 3.0))
    steps = int(math.ceil(T / dt))
    dtg = torch.tensor([T / steps], dtype=torch.float64, device="cuda")
    ug = torch.tensor(u0.reshape(S.ncomp, -1), device="cuda")
    mg = torch.tensor(m0.reshape(2, S.ncomp, -1), device="cuda")
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    for _ in range(steps):
        al = S.max_wavespeed(ug)
        S.stage(0, dtg, al, ug, mg, u1, m1)
        S.stage(1, dtg, al, u1, m1, u2, m2)
        S.stage(2, dtg, al, u2, m2, ug, mg)
    torch.cuda.synchronize()
    e = np.abs(ug.cpu().numpy()[0] - ue[0].reshape(-1))
    S.close()
    return e.max(), e.mean()


def test_2d_accuracy_tables_of_section_3_1():
    """The HWENO-U rows of the 2D accuracy tables (Examples 3.3 and 3.4),
    recomputed to the final times: 2D Burgers on [0, 4]^2 to T = 0.5/pi and
    2D Euler to T = 2 on one period, [0, 2]^2, of its solution (the printed
    errors are those of that domain; see the readings).  Every error lies
    within a factor 3 of the printed one, and within 10% on the meshes where
    the printed errors are asymptotic (measured: 0.2-3% for Euler at every
    mesh, and for Burgers from 160^2 on)."""
    print("[gpu] 2D accuracy tables", flush=True)
    cases = [("burgers2d", "burgers", n, 4.0, 0.5 / math.pi, 1.5, n >= 160)
             for n in (40, 80, 120, 160, 200, 240)]
    cases += [("euler2d", "euler", n, 2.0, 2.0, 1.0 + math.sqrt(1.4 / 0.8), True)
              for n in (40, 80, 120, 160)]
    for name, eq, n, L, T, ab, tight in cases:
        paper = _table(name)[n]
        got = _run_2d_table(eq, n, L, T, ab)
        ratio = [got[i] / paper[i] for i in range(2)]
        print(f"[gpu]   {name} {n}: Linf {got[0]:.3e} (paper {paper[0]:.2e}), "
              f"L1 {got[1]:.3e} (paper {paper[1]:.2e})", flush=True)
        band = 1.1 if tight else 3.0
        assert all(1.0 / band < r < band for r in ratio), (name, n, got, paper)


def _run_1d_table(eq, n):
    """FP64 run to the final time with dt = CFL dx^(5/3) / a, CFL 0.6;
    returns (L-inf, L1) of the average error and (L-inf, L1) of the moment
    error (Burgers)."""
    if eq == "euler":
        u0, m0 = W.euler_1d_sine(n)
        ue, ve = W.euler_1d_sine(n, t=2.0)
        L, T, ab = 2.0, 2.0, 1.0 + math.sqrt(1.4 / 0.8)
    else:
        u0, m0 = W.burgers_1d_initial(n)
        T = 0.5 / math.pi
        ue, ve = W.burgers_1d_exact_moments(n, T)
        L, ab = 2.0, 1.5
    S = H.Solver(1, eq, [H.make_inst(n, 1, (0.0, L))])
    dt = 0.6 * (L / n) ** (5.0 / 3.0) / ab
    steps = int(math.ceil(T / dt))
    dtg = torch.tensor([T / steps], dtype=torch.float64, device="cuda")
    ug, mg = torch.tensor(u0, device="cuda"), torch.tensor(m0, device="cuda")
    u1, m1 = S.empty_state()
    u2, m2 = S.empty_state()
    for _ in range(steps):
        al = S.max_wavespeed(ug)
        S.stage(0, dtg, al, ug, mg, u1, m1)
        S.stage(1, dtg, al, u1, m1, u2, m2)
        S.stage(2, dtg, al, u2, m2, ug, mg)
    torch.cuda.synchronize()
    e = np.abs(ug.cpu().numpy()[0] - ue[0])
    ev = np.abs(mg.cpu().numpy()[0, 0] - ve[0, 0])
    S.close()
    return (e.max(), e.mean()), (ev.max(), ev.mean())


def test_1d_accuracy_tables_of_section_3_1():
    """The HWENO-U rows of the 1D accuracy tables (Examples 3.1 and 3.2,
    and the first-moment errors of Example 3.1), recomputed on the GPU from
    80 cells on (40 cells is pre-asymptotic: 2-7 times the printed errors):
    within a factor 2 at 80 and 120 cells; from 160 cells on the L1 errors
    within 10% (measured 0.96-1.04) and the L-inf errors within a factor 1.4
    (measured 0.93-1.38)."""
    print("[gpu] 1D accuracy tables", flush=True)
    for eq, names in (("burgers", ("burgers1d", "burgers1d_v")), ("euler", ("euler1d",))):
        for n in (80, 120, 160, 200, 240):
            got = _run_1d_table(eq, n)
            for name, g in zip(names, got):
                paper = _table(name)[n]
                r = [g[i] / paper[i] for i in range(2)]
                print(f"[gpu]   {name} {n}: Linf {g[0]:.3e} (paper {paper[0]:.2e}), "
                      f"L1 {g[1]:.3e} (paper {paper[1]:.2e})", flush=True)
                bands = (1.4, 1.1) if n >= 160 else (2.0, 2.0)
                assert all(1.0 / b < x < b for x, b in zip(r, bands)), (name, n, r)
