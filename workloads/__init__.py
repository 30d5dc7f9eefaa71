"""Seeded synthetic inputs for the HWENO-U hot path.

This module holds problem set-up only -- initial conditions, their cell
averages and first-order moments, exact solutions and seeded random data --
and none of the scheme's arithmetic.  It is the one module that both the GPU
path's callers (tests, benchmark) and the CPU oracle's callers use.

Moments follow the paper's definitions (Section 2.1 / 2.2):
  u_i = (1/dx) int_{I_i} u dx,   v_i = (1/dx) int_{I_i} u (x - x_i)/dx dx,
  w_ij = (1/(dx dy)) int_{I_ij} u (y - y_j)/dy dx dy,
computed in closed form where one exists and otherwise with a Gauss-Legendre
rule per cell (q points per direction; every discontinuity of the seeded
data is placed on a cell face, so the integrand is smooth inside each cell).

Array layout: ubar [ncomp, n] (1D) or [ncomp, ny, nx] (2D, x fastest);
mom [dim, ncomp, ...] with mom[0] = x moments, mom[1] = y moments.
"""
import math

import numpy as np

GAS_GAMMA = 1.4


# ----------------------------------------------------------------------------
# generic quadrature of cell moments
# ----------------------------------------------------------------------------

def _gl(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * x, 0.5 * w  # nodes/weights on [-1/2, 1/2], weights sum to 1


def cell_moments_1d(func, a, b, n, q=8):
    """ubar, vbar of func over n uniform cells of [a, b].

    func(x) -> array of shape [ncomp, *x.shape] (or x.shape for a scalar)."""
    dx = (b - a) / n
    xc = a + (np.arange(n) + 0.5) * dx
    xi, w = _gl(q)
    X = xc[:, None] + dx * xi[None, :]
    F = np.asarray(func(X), dtype=np.float64)
    scalar = F.ndim == 2
    if scalar:
        F = F[None]
    ubar = np.einsum("knq,q->kn", F, w)
    vbar = np.einsum("knq,q->kn", F, w * xi)
    return ubar, vbar[None]


def cell_moments_2d(func, domain, nx, ny, q=4, rows_per_chunk=256):
    """ubar [ncomp, ny, nx], mom [2, ncomp, ny, nx] of func over a uniform grid."""
    a, b, c, d = domain
    dx, dy = (b - a) / nx, (d - c) / ny
    xi, w = _gl(q)
    xc = a + (np.arange(nx) + 0.5) * dx
    ubar = None
    for j0 in range(0, ny, rows_per_chunk):
        j1 = min(ny, j0 + rows_per_chunk)
        yc = c + (np.arange(j0, j1) + 0.5) * dy
        X = xc[None, :, None, None] + dx * xi[None, None, :, None]
        Y = yc[:, None, None, None] + dy * xi[None, None, None, :]
        X, Y = np.broadcast_arrays(X, Y)  # [rows, nx, qx, qy]
        F = np.asarray(func(X, Y), dtype=np.float64)
        if F.ndim == 4:
            F = F[None]
        if ubar is None:
            nc = F.shape[0]
            ubar = np.empty((nc, ny, nx))
            mom = np.empty((2, nc, ny, nx))
        ubar[:, j0:j1] = np.einsum("kjiab,a,b->kji", F, w, w)
        mom[0, :, j0:j1] = np.einsum("kjiab,a,b->kji", F, w * xi, w)
        mom[1, :, j0:j1] = np.einsum("kjiab,a,b->kji", F, w, w * xi)
    return ubar, mom


def prim_to_cons(rho, vel, p, gas_gamma=GAS_GAMMA):
    """Conserved variables (rho, rho*u[, rho*v], E) from primitives."""
    q2 = sum(v * v for v in vel)
    E = p / (gas_gamma - 1.0) + 0.5 * rho * q2
    return np.stack([rho] + [rho * v for v in vel] + [E])


# ----------------------------------------------------------------------------
# 1D workloads
# ----------------------------------------------------------------------------

def sine_1d(n, a=0.0, b=2.0, shift=0.0, offset=0.0):
    """Cell moments of offset + sin(pi (x - shift)), in closed form."""
    dx = (b - a) / n
    xl = a + np.arange(n) * dx
    xr = xl + dx
    xc = 0.5 * (xl + xr)
    k = math.pi
    # int sin(k(x-s)) dx = -cos(k(x-s))/k
    F0 = lambda x: -np.cos(k * (x - shift)) / k
    # int sin(k(x-s)) (x - xc) dx = -(x-xc) cos(k(x-s))/k + sin(k(x-s))/k^2
    F1 = lambda x: -(x - xc) * np.cos(k * (x - shift)) / k + np.sin(k * (x - shift)) / k ** 2
    ubar = offset + (F0(xr) - F0(xl)) / dx
    vbar = (F1(xr) - F1(xl)) / dx ** 2
    return ubar[None], vbar[None, None]


def advection_sine_1d(n=200):
    """Linear advection u_t + u_x = 0 on [0, 2], u0 = sin(pi x)."""
    return sine_1d(n, 0.0, 2.0)


def burgers_1d_initial(n):
    """Burgers accuracy test (Example 3.1): u0 = 0.5 + sin(pi x) on [0, 2]."""
    return sine_1d(n, 0.0, 2.0, offset=0.5)


def burgers_1d_exact(x, t):
    """Exact smooth solution of u_t + (u^2/2)_x = 0, u0 = 0.5 + sin(pi x)."""
    u = 0.5 + np.sin(np.pi * x)
    for _ in range(60):  # Newton on u - u0(x - u t) = 0
        arg = np.pi * (x - u * t)
        g = u - 0.5 - np.sin(arg)
        dg = 1.0 + np.pi * t * np.cos(arg)
        u = u - g / dg
    return u


def burgers_1d_exact_moments(n, t, q=8):
    return cell_moments_1d(lambda x: burgers_1d_exact(x, t), 0.0, 2.0, n, q)


def euler_1d_sine(n, t=0.0, gas_gamma=GAS_GAMMA):
    """Euler accuracy test (Example 3.2): rho = 1 + 0.2 sin(pi (x - t)), u = p = 1
    on [0, 2]; closed-form moments."""
    ub, vb = sine_1d(n, 0.0, 2.0, shift=t)
    rho = 1.0 + 0.2 * ub[0]
    rv = 0.2 * vb[0, 0]
    ubar = np.stack([rho, rho * 1.0, 1.0 / (gas_gamma - 1.0) + 0.5 * rho])
    vbar = np.stack([rv, rv, 0.5 * rv])
    return ubar, vbar[None]


def euler_1d_shocktube(n, seed, n_interfaces=16, gas_gamma=GAS_GAMMA, a=0.0, b=1.0):
    """Seeded piecewise-constant Euler states on [a, b] with a density wave.

    n_interfaces sorted U(0,1) positions (snapped to the nearest face) split
    the domain into n_interfaces+1 pieces with rho_k ~ U[0.125, 1],
    u_k ~ U[-1, 1], p_k ~ U[0.1, 1]; the density is rho_k (1 + 0.2 sin 5x).
    Moments are exact (sin integrals)."""
    rng = np.random.default_rng(seed)
    pos = np.sort(rng.uniform(0.0, 1.0, n_interfaces))
    ns = n_interfaces + 1
    rho_k = rng.uniform(0.125, 1.0, ns)
    u_k = rng.uniform(-1.0, 1.0, ns)
    p_k = rng.uniform(0.1, 1.0, ns)
    faces = np.clip(np.rint(pos * n).astype(np.int64), 0, n)
    piece = np.searchsorted(faces, np.arange(n), side="right")
    dx = (b - a) / n
    xl = a + np.arange(n) * dx
    xr = xl + dx
    xc = 0.5 * (xl + xr)
    kk = 5.0
    F0 = lambda x: -np.cos(kk * x) / kk
    F1 = lambda x: -(x - xc) * np.cos(kk * x) / kk + np.sin(kk * x) / kk ** 2
    s_avg = (F0(xr) - F0(xl)) / dx
    s_mom = (F1(xr) - F1(xl)) / dx ** 2
    r, u, p = rho_k[piece], u_k[piece], p_k[piece]
    rho_avg = r * (1.0 + 0.2 * s_avg)
    rho_mom = r * 0.2 * s_mom
    ubar = np.stack([rho_avg, rho_avg * u, p / (gas_gamma - 1.0) + 0.5 * u * u * rho_avg])
    vbar = np.stack([rho_mom, rho_mom * u, 0.5 * u * u * rho_mom])
    return ubar, vbar[None]


def euler_1d_riemann(n, left, right, x0, a, b, gas_gamma=GAS_GAMMA):
    """Two-state Riemann data (rho, u, p) with the jump on the face nearest x0."""
    face = int(round((x0 - a) / (b - a) * n))
    idx = np.arange(n)
    st = np.where(idx[None, :] < face, np.array(left)[:, None], np.array(right)[:, None])
    ubar = prim_to_cons(st[0], [st[1]], st[2], gas_gamma)
    return ubar, np.zeros((1,) + ubar.shape)


def _piecewise_prim(n, a, b, pieces, gas_gamma=GAS_GAMMA):
    """Cell data of piecewise-constant primitive states (rho, u, p) with every
    jump on a cell face: pieces = [(x_end, (rho, u, p)), ...]."""
    xc = a + (np.arange(n) + 0.5) * (b - a) / n
    st = np.empty((3, n))
    lo = a
    for x_end, prim in pieces:
        sel = (xc > lo) & (xc < x_end)
        st[:, sel] = np.array(prim, dtype=np.float64)[:, None]
        lo = x_end
    ubar = prim_to_cons(st[0], [st[1]], st[2], gas_gamma)
    return ubar, np.zeros((1,) + ubar.shape)


# 1D shock problems of Section 3.2: name -> (cells, domain, boundary, final time)
SHOCK_SUITE_1D = {
    "lax": (200, (-0.5, 0.5), "transmissive", 0.16),
    "blast": (800, (0.0, 1.0), "reflective", 0.038),
    "shu_osher": (400, (-5.0, 5.0), "transmissive", 1.8),
    "double_rarefaction": (400, (-1.0, 1.0), "transmissive", 0.6),
    "sedov": (801, (-2.0, 2.0), "transmissive", 0.001),
}
LAX_STATES = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def shock_suite_1d(name, n=None):
    """Initial cell averages and moments of a 1D shock problem of Section 3.2
    (Lax, interacting blast waves, Shu-Osher, double rarefaction, Sedov).
    The Sedov problem puts the energy 3.2e6 / dx into the centre cell of an
    odd number of cells (801; the paper's 800 cells have no centre cell)."""
    n0, (a, b), _, _ = SHOCK_SUITE_1D[name]
    n = n0 if n is None else n
    if name == "lax":
        return _piecewise_prim(n, a, b, [(0.0, LAX_STATES[0]), (b, LAX_STATES[1])])
    if name == "blast":
        return _piecewise_prim(n, a, b, [(0.1, (1.0, 0.0, 1000.0)), (0.9, (1.0, 0.0, 0.01)),
                                         (b, (1.0, 0.0, 100.0))])
    if name == "double_rarefaction":
        return _piecewise_prim(n, a, b, [(0.0, (7.0, -1.0, 0.2)), (b, (7.0, 1.0, 0.2))])
    if name == "shu_osher":
        def f(X):
            left = X < -4.0
            rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * X))
            u = np.where(left, 2.629369, 0.0)
            p = np.where(left, 10.333333, 1.0)
            return prim_to_cons(rho, [u], p)
        return cell_moments_1d(f, a, b, n)
    if name == "sedov":
        assert n % 2 == 1, "the Sedov problem needs a centre cell"
        dx = (b - a) / n
        ubar = np.zeros((3, n))
        ubar[0] = 1.0
        ubar[2] = 1e-12
        ubar[2, n // 2] = 3200000.0 / dx
        return ubar, np.zeros((1, 3, n))
    raise ValueError(name)


def riemann_exact(left, right, xi, gas_gamma=GAS_GAMMA, tol=1e-14):
    """Exact solution of the 1D Euler Riemann problem (primitive states
    (rho, u, p) left and right of x = 0) at similarity coordinates
    xi = x / t: the star pressure from Newton's method on the pressure
    function, then sampling of the wave pattern (two shocks or rarefactions
    around a contact; no vacuum).  Returns rho, u, p arrays."""
    g = gas_gamma
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    assert 2.0 / (g - 1.0) * (cl + cr) > ur - ul, "vacuum is generated"

    def fk(p, rk, pk, ck):
        if p > pk:  # shock
            A, B = 2.0 / ((g + 1.0) * rk), (g - 1.0) / (g + 1.0) * pk
            q = math.sqrt(A / (p + B))
            return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
        r = (p / pk) ** ((g - 1.0) / (2.0 * g))  # rarefaction
        return 2.0 * ck / (g - 1.0) * (r - 1.0), r / (rk * ck)

    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, cl)
        f2, d2 = fk(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p_new = max(p - dp, 1e-14)
        if abs(p_new - p) <= tol * (p_new + p):
            p = p_new
            break
        p = p_new
    us = 0.5 * (ul + ur) + 0.5 * (fk(p, rr, pr, cr)[0] - fk(p, rl, pl, cl)[0])
    xi = np.asarray(xi, dtype=np.float64)
    rho, u, pp = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    for side, (rk, uk, pk, ck, sgn) in enumerate(((rl, ul, pl, cl, -1.0), (rr, ur, pr, cr, 1.0))):
        sel = xi <= us if side == 0 else xi > us
        x = xi[sel]
        if p > pk:  # shock moving away from the contact
            rs = rk * ((p / pk + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * p / pk + 1.0))
            S = uk + sgn * ck * math.sqrt((g + 1.0) / (2.0 * g) * p / pk + (g - 1.0) / (2.0 * g))
            out = sgn * (x - S) > 0
            rho[sel] = np.where(out, rk, rs)
            u[sel] = np.where(out, uk, us)
            pp[sel] = np.where(out, pk, p)
        else:  # rarefaction fan
            rs = rk * (p / pk) ** (1.0 / g)
            cs = ck * (p / pk) ** ((g - 1.0) / (2.0 * g))
            head, tail = uk + sgn * ck, us + sgn * cs
            r_out = sgn * (x - head) > 0
            r_in = sgn * (x - tail) < 0
            fan_u = 2.0 / (g + 1.0) * (-sgn * ck + (g - 1.0) / 2.0 * uk + x)
            fan_c = sgn * (fan_u - x)
            fan_rho = rk * np.abs(fan_c / ck) ** (2.0 / (g - 1.0))
            fan_p = pk * np.abs(fan_c / ck) ** (2.0 * g / (g - 1.0))
            rho[sel] = np.where(r_out, rk, np.where(r_in, rs, fan_rho))
            u[sel] = np.where(r_out, uk, np.where(r_in, us, fan_u))
            pp[sel] = np.where(r_out, pk, np.where(r_in, p, fan_p))
    return rho, u, pp


def riemann_exact_averages(left, right, n, a, b, x0, t, samples=64, gas_gamma=GAS_GAMMA):
    """Cell averages of the exact Riemann density at time t (midpoint rule
    with `samples` points per cell)."""
    dx = (b - a) / n
    x = a + (np.arange(n)[:, None] + (np.arange(samples)[None, :] + 0.5) / samples) * dx
    rho, _, _ = riemann_exact(left, right, (x - x0) / t, gas_gamma)
    return rho.mean(axis=1)


# ----------------------------------------------------------------------------
# 2D workloads
# ----------------------------------------------------------------------------

def burgers_2d_initial(n, q=4):
    """Example 3.3: u0 = 0.5 + sin(pi (x + y)/2) on [0, 4]^2."""
    f = lambda X, Y: 0.5 + np.sin(np.pi * (X + Y) / 2.0)
    return cell_moments_2d(f, (0.0, 4.0, 0.0, 4.0), n, n, q)


def burgers_2d_exact_moments(n, t, q=6):
    """Exact solution of Example 3.3 at time t: it is the 1D solution of
    u_s + (u^2/2)_s = 0 along s = (x + y)/2 with the same profile."""
    f = lambda X, Y: burgers_1d_exact(0.5 * (X + Y), t)
    return cell_moments_2d(f, (0.0, 4.0, 0.0, 4.0), n, n, q)


def euler_2d_sine(n, t=0.0, gas_gamma=GAS_GAMMA, q=4, L=4.0):
    """Example 3.4: rho = 1 + 0.2 sin(pi (x + y - 2t)), u = v = p = 1 on
    [0, L]^2 (the text's L = 4; the printed errors belong to one period,
    L = 2, of the same solution)."""
    def f(X, Y):
        rho = 1.0 + 0.2 * np.sin(np.pi * (X + Y - 2.0 * t))
        one = np.ones_like(rho)
        return prim_to_cons(rho, [one, one], one, gas_gamma)
    return cell_moments_2d(f, (0.0, L, 0.0, L), n, n, q)


def vortex_factors(X, Y, xc, yc, strength, gas_gamma=GAS_GAMMA):
    """Isentropic vortex perturbation: (du, dv, temperature factor)."""
    xb, yb = X - xc, Y - yc
    r2 = xb * xb + yb * yb
    e = np.exp(0.5 * (1.0 - r2))
    du = strength / (2.0 * np.pi) * e * (-yb)
    dv = strength / (2.0 * np.pi) * e * xb
    T = 1.0 - (gas_gamma - 1.0) * strength ** 2 / (8.0 * gas_gamma * np.pi ** 2) * e * e
    return du, dv, T


def quadrant_states(seed, vel_range=0.5):
    """Seeded four-quadrant Riemann states (rho, u, v, p), shape [4, 4];
    quadrant index = (y >= mid) * 2 + (x >= mid)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 1.5, 4)
    p = rng.uniform(0.03, 1.5, 4)
    u = rng.uniform(-vel_range, vel_range, 4)
    v = rng.uniform(-vel_range, vel_range, 4)
    return np.stack([rho, u, v, p], axis=1)


def euler_2d_vortex_quadrant(nx, ny=None, seed=3000, L=10.0, strength=5.0, gas_gamma=GAS_GAMMA,
                             q=4, vel_range=0.5):
    """Seeded four-quadrant Riemann data on [0, L]^2 (periodic) times an
    isentropic vortex of the given strength centred at (L/4, L/4).  Quadrant
    splits at x = L/2 and y = L/2 are on cell faces for even nx, ny."""
    ny = nx if ny is None else ny
    st = quadrant_states(seed, vel_range)
    mid = 0.5 * L

    def f(X, Y):
        qd = (Y >= mid).astype(np.int64) * 2 + (X >= mid).astype(np.int64)
        rho, u, v, p = (st[qd, k] for k in range(4))
        du, dv, T = vortex_factors(X, Y, 0.25 * L, 0.25 * L, strength, gas_gamma)
        rho = rho * T ** (1.0 / (gas_gamma - 1.0))
        p = p * T ** (gas_gamma / (gas_gamma - 1.0))
        return prim_to_cons(rho, [u + du, v + dv], p, gas_gamma)

    # cell centres of a cell never straddle the quadrant split when the split is
    # on a face, so evaluating the quadrant from the quadrature node is exact.
    return cell_moments_2d(f, (0.0, L, 0.0, L), nx, ny, q)


def euler_2d_vortex(nx, t=0.0, L=10.0, strength=5.0, mean=(1.0, 1.0), gas_gamma=GAS_GAMMA,
                    q=4):
    """Smooth isentropic vortex on the uniform state rho = p = 1 moving with
    `mean` on [0, L]^2; the exact solution at t is the translated vortex."""
    def f(X, Y):
        xc = (0.5 * L + mean[0] * t) % L
        yc = (0.5 * L + mean[1] * t) % L
        # nearest periodic image of the centre
        Xs = (X - xc + 0.5 * L) % L - 0.5 * L
        Ys = (Y - yc + 0.5 * L) % L - 0.5 * L
        du, dv, T = vortex_factors(Xs, Ys, 0.0, 0.0, strength, gas_gamma)
        rho = T ** (1.0 / (gas_gamma - 1.0))
        p = T ** (gas_gamma / (gas_gamma - 1.0))
        return prim_to_cons(rho, [mean[0] + du, mean[1] + dv], p, gas_gamma)
    return cell_moments_2d(f, (0.0, L, 0.0, L), nx, nx, q)


# ----------------------------------------------------------------------------
# batches
# ----------------------------------------------------------------------------

def log_uniform_sizes(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def batch_1d_euler(count=512, lo=256, hi=65536, seed=4000):
    """Independent 1D Euler shock-tube instances with log-uniform sizes.
    Returns (sizes, [(ubar, mom), ...]); instance k uses seed + 1 + k."""
    sizes = log_uniform_sizes(count, lo, hi, seed)
    return sizes, [euler_1d_shocktube(int(n), seed + 1 + k) for k, n in enumerate(sizes)]


def batch_2d_euler(count=64, lo=256, hi=1024, seed=5000, q=2):
    """Independent 2D Euler vortex+quadrant instances with log-uniform
    square sides (rounded to even).  Instance k uses seed + 1 + k."""
    sides = log_uniform_sizes(count, lo, hi, seed)
    sides = sides + (sides % 2)
    return sides, [euler_2d_vortex_quadrant(int(n), seed=seed + 1 + k, q=q)
                   for k, n in enumerate(sides)]


def random_smooth_1d(n, ncomp, seed, positive_euler=False, gas_gamma=GAS_GAMMA):
    """Small random periodic data for parity tests (few Fourier modes)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(ncomp, 4))
    ph = rng.uniform(0, 2 * np.pi, size=(ncomp, 4))

    def f(x):
        out = []
        for k in range(ncomp):
            s = sum(a[k, m] / (m + 1) * np.sin(np.pi * (m + 1) * x + ph[k, m]) for m in range(4))
            out.append(s)
        out = np.stack(out)
        if positive_euler:
            rho = 1.0 + 0.3 * np.tanh(out[0])
            u = 0.5 * np.tanh(out[1])
            p = 1.0 + 0.3 * np.tanh(out[2])
            return prim_to_cons(rho, [u], p, gas_gamma)
        return out
    return cell_moments_1d(f, 0.0, 2.0, n)
