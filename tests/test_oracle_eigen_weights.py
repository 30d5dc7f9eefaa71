"""Pins of the oracle's characteristic basis and of its 2D weight conventions.

* The Euler eigenvector basis that the reconstruction projects with
  (Remark 2.2, the local characteristic decomposition; the basis is reading
  R5) must diagonalise the flux Jacobian: A(U) R = R diag(u_n - c, u_n, u_n,
  u_n + c).  The Jacobian is built here by complex-step differentiation of an
  Euler flux written in this file, not by the oracle's own flux.
* The 2D u_ave of Eq. (2.22) is taken over the five-cell cross {2, 4, 5, 6, 8}:
  by the remark after Eq. (2.11), u_ave = 0 turns the nonlinear weights into
  the linear ones, so vanishing cross averages (corners non-zero) must give
  exactly the linear-weight moment modification, and any one non-zero cross
  cell must not.
* The 2D tau of Eq. (2.21) averages its four differences as the 1D tau of
  Eq. (2.10) averages its two: on y-constant quadratic data (reproduced
  exactly by both quartics, so both give the same smoothness indicators for
  a square mesh) whose averages satisfy |u_4| + |u_6| = 2 |u_5| (so that the
  five-cell 2D u_ave equals the three-cell 1D one), the 2D weights reduce to
  the 1D ones, and the 2D v^ equals the 1D v^ (with the 1D linear weight
  2 gamma_low, which the reduction pairs with the 2D gamma_low).

Every pin is shown to fail on an oracle built with the matching planted
mistake (ORACLE_PLANT in hwenou_oracle.c).
"""
import numpy as np
import pytest

from oracle import build as obuild
from oracle import driver
from oracle.driver import Problem

GAMMA = 1.4


# ---------------------------------------------------------------------------
# Euler flux and its Jacobian, written here
# ---------------------------------------------------------------------------

def _flux(U, dim, direction, gamma=GAMMA):
    """Euler flux in direction `direction` of the conserved state U
    (rho, rho u[, rho v], E); complex-safe for complex-step derivatives."""
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(dim)]
    E = U[dim + 1]
    p = (gamma - 1.0) * (E - 0.5 * rho * sum(v * v for v in vel))
    un = vel[direction]
    F = [rho * un]
    for d in range(dim):
        F.append(U[1 + d] * un + (p if d == direction else 0.0))
    F.append(un * (E + p))
    return np.array(F)


def _jacobian(U, dim, direction):
    n = dim + 2
    J = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        Uc = np.array(U, dtype=np.complex128)
        Uc[k] += 1j * h
        J[:, k] = _flux(Uc, dim, direction).imag / h
    return J


def _states(seed, dim, count=12):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        rho = rng.uniform(0.05, 5.0)
        vel = rng.uniform(-3.0, 3.0, dim)
        p = rng.uniform(0.01, 10.0)
        E = p / (GAMMA - 1.0) + 0.5 * rho * float(vel @ vel)
        out.append(np.array([rho, *(rho * vel), E]))
    return out


def _eigen_residual(dim, direction, seed):
    """max over states of |A R - R Lambda| / (|A| |R|), and of |L R - I|."""
    P = Problem(dim, "euler", 8 if dim == 1 else (8, 8), (0, 1) if dim == 1 else (0, 1, 0, 1))
    worst, worst_inv = 0.0, 0.0
    for U in _states(seed, dim):
        R, L = P.eigvecs(U, direction)
        rho = U[0]
        vel = U[1:dim + 1] / rho
        p = (GAMMA - 1.0) * (U[dim + 1] - 0.5 * rho * float(vel @ vel))
        c = np.sqrt(GAMMA * p / rho)
        un = vel[direction]
        lam = [un - c, un, un + c] if dim == 1 else [un - c, un, un, un + c]
        A = _jacobian(U, dim, direction)
        res = np.abs(A @ R - R @ np.diag(lam)).max()
        worst = max(worst, res / (np.abs(A).max() * np.abs(R).max()))
        worst_inv = max(worst_inv, np.abs(L @ R - np.eye(dim + 2)).max())
    return worst, worst_inv


@pytest.mark.parametrize("dim,direction", [(1, 0), (2, 0), (2, 1)])
def test_eigenvectors_diagonalise_the_flux_jacobian(dim, direction):
    res, inv = _eigen_residual(dim, direction, seed=900 + 10 * dim + direction)
    assert res <= 1e-14, res
    assert inv <= 1e-13, inv


@pytest.mark.parametrize("dim,direction", [(1, 0), (2, 0), (2, 1)])
def test_eigenvector_normalisation(dim, direction):
    """Reading R5 fixes one normalisation of the basis: unit density entry in
    the acoustic and entropy columns; in 2D the shear column is the unit
    tangential momentum plus the tangential velocity in the energy."""
    P = Problem(dim, "euler", 8 if dim == 1 else (8, 8), (0, 1) if dim == 1 else (0, 1, 0, 1))
    for U in _states(77, dim, 4):
        R, _ = P.eigvecs(U, direction)
        vel = U[1:dim + 1] / U[0]
        if dim == 1:
            assert np.array_equal(R[0], [1.0, 1.0, 1.0])
            assert R[1, 1] == vel[0] and R[2, 1] == pytest.approx(0.5 * vel[0] ** 2, rel=1e-15)
        else:
            n, t = 1 + direction, 2 - direction
            assert np.array_equal(R[0], [1.0, 1.0, 0.0, 1.0])
            assert R[n, 2] == 0.0 and R[t, 2] == 1.0
            assert R[3, 2] == pytest.approx(vel[1 - direction], rel=1e-15)
            assert R[3, 1] == pytest.approx(0.5 * float(vel @ vel), rel=1e-15)


@pytest.fixture(scope="module")
def planted(tmp_path_factory):
    """Oracle libraries with one planted mistake each (ORACLE_PLANT)."""
    d = tmp_path_factory.mktemp("planted")
    return {k: driver.load(obuild.build(out=str(d / f"liboracle_plant{k}.so"), plant=k))
            for k in (1, 2, 3)}


def test_eigenvector_pin_fails_on_a_planted_wrong_column(planted):
    """Negative control: q^2 instead of q^2/2 in the entropy column."""
    with driver.using(planted[1]):
        for dim, direction in [(1, 0), (2, 0), (2, 1)]:
            res, _ = _eigen_residual(dim, direction, seed=900 + 10 * dim + direction)
            assert res > 1e-3, (dim, direction, res)


# ---------------------------------------------------------------------------
# 2D u_ave: the five-cell cross
# ---------------------------------------------------------------------------

def _vhat_target_2d(u_centre3x3, mom_seed, weights):
    """v^ and w^ of the centre cell of a 5x5 outflow grid whose 3x3 block
    around the centre holds the given averages (others zero), with seeded
    moments; scalar advection (the weights do not depend on the flux)."""
    n = 5
    u = np.zeros((1, n, n))
    u[0, 1:4, 1:4] = u_centre3x3
    rng = np.random.default_rng(mom_seed)
    m = rng.uniform(-0.3, 0.3, (2, 1, n, n))
    P = Problem(2, "advection", (n, n), (0, 5, 0, 5), bc="transmissive", adv=(1.0, 0.5),
                weights=weights)
    _, _, mh = P.rhs(u, m, [1.0, 0.5])
    return mh[:, 0, 2, 2]


def _cross_pin_failures():
    """Cells of the 3x3 stencil for which the pin's expectation fails:
    non-zero cross averages must move v^/w^ away from the linear-weight
    values, non-zero corners alone must not."""
    bad = []
    rng = np.random.default_rng(5)
    corners = np.zeros((3, 3))
    for b, a in [(0, 0), (0, 2), (2, 0), (2, 2)]:
        corners[b, a] = rng.uniform(0.5, 1.5) * rng.choice([-1, 1])
    lin = _vhat_target_2d(corners, 11, "linear")
    si = _vhat_target_2d(corners, 11, "scale_invariant")
    if np.abs(si - lin).max() > 1e-13 * np.abs(lin).max():
        bad.append("corners")
    for b, a in [(0, 1), (1, 0), (1, 1), (1, 2), (2, 1)]:
        g = corners.copy()
        g[b, a] = 0.9
        lin = _vhat_target_2d(g, 11, "linear")
        si = _vhat_target_2d(g, 11, "scale_invariant")
        if np.abs(si - lin).max() < 1e-4 * np.abs(lin).max():
            bad.append((b, a))
    return bad


def test_2d_u_ave_is_taken_over_the_five_cell_cross():
    assert _cross_pin_failures() == []


def test_u_ave_pin_fails_on_a_planted_nine_cell_average(planted):
    with driver.using(planted[3]):
        assert "corners" in _cross_pin_failures()


# ---------------------------------------------------------------------------
# 2D tau: the mean of four differences reduces to the 1D mean of two
# ---------------------------------------------------------------------------

def _quadratic_data(n, i0, C):
    """Cell averages and first moments (unit cells) of the quadratic
    p(x) = 25C/24 + C s - C s^2 / 2, s = x - x_{i0}, whose averages on cells
    i0-1, i0, i0+1 are -C/2, C, 3C/2 (slopes 3C/2 and C/2)."""
    a, b, c = 25.0 * C / 24.0, C, -0.5 * C
    k = np.arange(n) - i0
    avg = a + b * k + c * (k * k + 1.0 / 12.0)
    mom = (b + 2.0 * c * k) / 12.0
    return avg, mom


def _tau_pin_gap(eps=1e-10):
    """|v^_2D - v^_1D| / |v^_1D| at the target cell, and the distance of the
    1D v^ from its linear-weight value (which shows the weights matter)."""
    n, i0, C = 8, 4, 0.7
    avg, mom = _quadratic_data(n, i0, C)
    gl = 1.0 / 400.0
    P1 = Problem(1, "advection", n, (0, n), bc="transmissive", adv=(1.0,), gamma_low=2 * gl,
                 eps=eps)
    _, _, mh1 = P1.rhs(avg[None], mom[None, None], [1.0])
    P1l = Problem(1, "advection", n, (0, n), bc="transmissive", adv=(1.0,), gamma_low=2 * gl,
                  eps=eps, weights="linear")
    _, _, mh1l = P1l.rhs(avg[None], mom[None, None], [1.0])
    ny = 4
    u2 = np.repeat(avg[None, None, :], ny, axis=1)
    m2 = np.zeros((2, 1, ny, n))
    m2[0, 0] = mom[None, :]
    P2 = Problem(2, "advection", (n, ny), (0, n, 0, ny),
                 bc=("transmissive", "transmissive", "periodic", "periodic"), adv=(1.0, 0.0),
                 gamma_low=gl, eps=eps)
    _, _, mh2 = P2.rhs(u2, m2, [1.0, 0.0])
    v1 = mh1[0, 0, i0]
    v2 = mh2[0, 0, :, i0]
    gap = float(np.abs(v2 - v1).max() / abs(v1))
    nonlin = float(abs(v1 - mh1l[0, 0, i0]) / abs(v1))
    return gap, nonlin, float(np.abs(mh2[1, 0, :, i0]).max())


def test_2d_tau_reduces_to_the_1d_tau():
    gap, nonlin, w_hat = _tau_pin_gap()
    assert 1e-3 < nonlin < 1.0, nonlin  # the nonlinear weights matter here
    assert gap <= 1e-13, gap
    assert w_hat <= 1e-15  # y-constant data: no y-moment


def test_tau_pin_fails_on_a_planted_divisor(planted):
    with driver.using(planted[2]):
        gap, _, _ = _tau_pin_gap()
    assert gap > 1e-4, gap


# ---------------------------------------------------------------------------
# per-interface projection: the Roe average and its bases
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def planted_iface(tmp_path_factory):
    d = tmp_path_factory.mktemp("planted_iface")
    return {k: driver.load(obuild.build(out=str(d / f"liboracle_plant{k}.so"), plant=k))
            for k in (4, 5)}


def _roe_residual(seed):
    """max over random state pairs and both 2D directions of
    |A(U_roe)(U_R - U_L) - (F(U_R) - F(U_L))| / |F(U_R) - F(U_L)|, and of
    |Roe(U, U) - U| / |U|."""
    P = Problem(2, "euler", (8, 8), (0, 1, 0, 1))
    states = _states(seed, 2, 16)
    worst, same = 0.0, 0.0
    for UL, UR in zip(states[::2], states[1::2]):
        Ur = P.roe_state(UL, UR)
        for direction in (0, 1):
            A = _jacobian(Ur, 2, direction)
            dF = _flux(UR, 2, direction) - _flux(UL, 2, direction)
            worst = max(worst, np.abs(A @ (UR - UL) - dF).max() / np.abs(dF).max())
        same = max(same, np.abs(P.roe_state(UL, UL) - UL).max() / np.abs(UL).max())
    return worst, same


def test_roe_average_linearises_the_flux():
    """The Roe average (the textbook property that defines it): the flux
    Jacobian at the averaged state maps the jump of the conserved variables
    onto the jump of the flux exactly, in both directions; and it is
    consistent, Roe(U, U) = U."""
    worst, same = _roe_residual(1300)
    assert worst <= 1e-13, worst
    assert same <= 1e-15, same


def test_roe_pin_fails_on_a_planted_enthalpy_mean(planted_iface):
    with driver.using(planted_iface[4]):
        worst, _ = _roe_residual(1300)
    assert worst > 1e-4, worst


def _blocks_case(seed, nx=16, ny=4, width=4):
    """y-constant data whose averages are constant on blocks of `width`
    columns (states within 5% of rho = p = 1 at rest, so that the weights
    stay away from the one-sided limits where every basis gives the same
    constant) and whose x-moments are random, up to 10% of the averages."""
    rng = np.random.default_rng(seed)
    u = np.zeros((4, ny, nx))
    for b in range(0, nx, width):
        rho, vx, vy, p = 1.0 + 0.05 * rng.uniform(-1, 1, 4) - np.array([0.0, 1.0, 1.0, 0.0])
        u[:, :, b:b + width] = np.array([rho, rho * vx, rho * vy,
                                         p / 0.4 + 0.5 * rho * (vx * vx + vy * vy)])[:, None, None]
    m = np.zeros((2, 4, ny, nx))
    m[0] = rng.uniform(-0.1, 0.1, (4, 1, nx)) * np.abs(u[:, :1, :])
    return u, m


def _iface_block_gap(seed=1400, width=4):
    """Largest relative F1 difference between the per-interface and the
    split schemes over the cells whose two x-interfaces lie inside a block
    of equal averages (there every interface basis is the cells' own one),
    and the smallest one over the cells next to a block edge."""
    u, m = _blocks_case(seed, width=width)
    nx = u.shape[2]
    out = {}
    for mode in (1, 3):
        P = Problem(2, "euler", (nx, u.shape[1]), (0, 10, 0, 2.5), char_decomp=mode)
        out[mode] = P.rhs(u, m, P.max_wavespeed(u))
    d = np.abs(out[3][0] - out[1][0]).max(axis=(0, 1)) / np.abs(out[1][0]).max()
    inner = [i for i in range(nx) if 0 < i % width < width - 1]
    edge = [i for i in range(nx) if i % width in (0, width - 1)]
    same_vhat = np.abs(out[3][2] - out[1][2]).max()
    return float(d[inner].max()), float(d[edge].min()), float(same_vhat)


def test_interface_bases_are_shared_by_both_sides():
    """Both sides of an interface are reconstructed in the basis of that
    interface (the Roe average of the two cells), and the interior values and
    v^, w^ in the cell's own one: wherever two neighbours have equal
    averages, their interface's basis is their own, so the per-interface
    scheme equals the split scheme at every cell whose two interfaces lie
    inside a block of equal averages (to rounding), differs next to the
    block edges, and has the same v^, w^ everywhere."""
    inner, edge, same_vhat = _iface_block_gap()
    assert inner <= 1e-12, inner  # measured 5e-15
    assert edge > 1e-6, edge  # measured 6e-5
    assert same_vhat == 0.0


def test_interface_pin_fails_on_planted_swapped_bases(planted_iface):
    with driver.using(planted_iface[5]):
        inner, _, _ = _iface_block_gap()
    assert inner > 1e-5, inner  # measured 1e-3
