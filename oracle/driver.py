"""Python driver of the HWENO-U CPU oracle.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark import this module.  It loads the plain-C
oracle (hwenou_oracle.c), hands it the operators derived exactly in
derive.py, and performs the modified SSP Runge-Kutta combination of
Eq. (2.13) (Section 2.1, Step 4; used unchanged in 2D, Section 2.2, Step 4):

  stage 0:  U1    = (u^n, v^n_hat) + dt F(U^n)
  stage 1:  U2    = 3/4 (u^n, v^n_hat) + 1/4 ((u1, v1_hat) + dt F(U1))
  stage 2:  U^n+1 = 1/3 (u^n, v^n_hat) + 2/3 ((u2, v2_hat) + dt F(U2))

where v_hat is the HWENO moment modification computed from the same
reconstruction as F.  The time step follows dt = CFL dx / alpha (1D) and
dt = CFL / (alpha_1/dx + alpha_2/dy) (2D), clipped at the final time, with
alpha the maximum wave speed over the cell averages of U^n.

State arrays: ubar [ncomp, n] or [ncomp, ny, nx]; mom [dim, ncomp, ...]
(mom[0] = x moments v, mom[1] = y moments w).
"""
import ctypes as C
import os

import numpy as np

from . import derive

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

EQ = {"advection": 0, "burgers": 1, "euler": 2}
WEIGHTS = {"scale_invariant": 0, "zq": 1, "linear": 2}
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
ERR_NONPHYSICAL = 4


class NonPhysicalState(RuntimeError):
    pass


class _Params(C.Structure):
    _fields_ = [("eq", C.c_int), ("ncomp", C.c_int), ("weights", C.c_int),
                ("char_decomp", C.c_int), ("adv_x", C.c_double), ("adv_y", C.c_double),
                ("gas_gamma", C.c_double), ("gamma_low", C.c_double), ("eps", C.c_double)]


_lib = None


def _flat(M):
    return np.ascontiguousarray(np.array(derive.as_float_rows(M), dtype=np.float64).ravel())


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build
        build.build()
    _lib = load(LIB_PATH)
    return _lib


def load(path):
    """Load a built oracle library and hand it the derived operators."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.oracle_rhs_1d.argtypes = [C.POINTER(_Params), C.c_int, C.c_double, C.c_int, C.c_int,
                                C.c_double, dp, dp, dp, dp, dp]
    L.oracle_rhs_2d.argtypes = [C.POINTER(_Params), C.c_int, C.c_int, C.c_double, C.c_double,
                                C.POINTER(C.c_int), dp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.oracle_max_wavespeed.argtypes = [C.POINTER(_Params), C.c_int, C.c_size_t, dp, dp]
    L.oracle_all_physical.argtypes = [C.POINTER(_Params), C.c_int, C.c_size_t, dp]
    L.oracle_num_threads.restype = C.c_int
    L.oracle_set_num_threads.argtypes = [C.c_int]
    L.oracle_eigvecs.argtypes = [C.POINTER(_Params), dp, C.c_int, C.c_int, dp, dp]
    L.oracle_roe_state.argtypes = [C.POINTER(_Params), dp, dp, C.c_int, dp]
    # hand in the exactly derived operators
    r1 = derive.recon_1d()
    keep = [_flat(r1["M0"]), _flat(r1["M1"]), _flat(r1["M2"]), _flat(derive.beta_gram_1d(4)),
            _flat(derive.beta_gram_1d(1)),
            np.array([float(v) for v in derive.q_row_1d(4)]),
            np.array([float(v) for v in derive.q_row_1d(1)])]
    L.oracle_set_ops_1d(*[a.ctypes.data_as(dp) for a in keep])
    r2 = derive.recon_2d()
    qv4, qw4 = derive.q_rows_2d(4)
    qv1, qw1 = derive.q_rows_2d(1)
    keep2 = [_flat(r2["M0"]), np.concatenate([_flat(M) for M in r2["Mm"]]),
             _flat(derive.beta_gram_2d(4)), _flat(derive.beta_gram_2d(1)),
             np.array([float(v) for v in qv4]), np.array([float(v) for v in qw4]),
             np.array([float(v) for v in qv1]), np.array([float(v) for v in qw1])]
    L.oracle_set_ops_2d(*[np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(dp)
                          for a in keep2])
    return L


class using:
    """Context manager: route every oracle call through another loaded
    library (a planted variant built by the tests), then restore."""

    def __init__(self, L):
        self.L = L

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = self.L
        return self.L

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    """Thread count of later oracle calls (timing only; results do not depend
    on it: every cell is computed independently)."""
    lib().oracle_set_num_threads(int(n))


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _char_mode(c):
    """True / 1: direction-split characteristic sweeps; False / 0:
    component-wise; 2 or 'single': one x-characteristic reconstruction for
    both directions; 3 or 'interface': split sweeps with the edge values at
    each interface in the characteristic variables of the Roe average of the
    two cells that share it (2D)."""
    if c == "single":
        return 2
    if c == "interface":
        return 3
    return int(c)


class Problem:
    """A single HWENO-U problem on a uniform periodic/transmissive grid.

    dim: 1 or 2.  eq: 'advection' | 'burgers' | 'euler'.
    n: number of cells (1D) or (nx, ny) (2D).  domain: (a, b) or (a, b, c, d).
    bc: 'periodic' | 'transmissive' | 'reflective' (Euler walls) or a tuple per side
        (x-lo, x-hi[, y-lo, y-hi]).
    char_decomp (Euler): True / 1 direction-split characteristic sweeps (the
        default), False / 0 component-wise, 2 / 'single' one reconstruction in
        x-characteristic variables for every output (2D), 3 / 'interface'
        split sweeps with interface (Roe-average) bases for the edge values
        (2D).
    """

    def __init__(self, dim, eq, n, domain, bc="periodic", gas_gamma=1.4, adv=(1.0, 1.0),
                 weights="scale_invariant", char_decomp=True, gamma_low=1.0 / 400.0,
                 eps=1e-10):
        self.dim = dim
        self.eq = eq
        if dim == 1:
            self.nx, self.ny = int(n), 1
            self.dx = (domain[1] - domain[0]) / self.nx
            self.dy = 1.0
        else:
            self.nx, self.ny = int(n[0]), int(n[1])
            self.dx = (domain[1] - domain[0]) / self.nx
            self.dy = (domain[3] - domain[2]) / self.ny
        self.domain = tuple(domain)
        if isinstance(bc, str):
            bc = (bc,) * (2 * dim)
        self.bc = tuple(BC[b] for b in bc)
        self.ncomp = 1 if eq != "euler" else dim + 2
        self.params = _Params(EQ[eq], self.ncomp, WEIGHTS[weights], _char_mode(char_decomp),
                              float(adv[0]), float(adv[1] if len(adv) > 1 else 0.0),
                              float(gas_gamma), float(gamma_low), float(eps))

    # -- shapes ---------------------------------------------------------------
    @property
    def shape(self):
        return (self.ncomp, self.nx) if self.dim == 1 else (self.ncomp, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny

    # -- operators ------------------------------------------------------------
    def max_wavespeed(self, ubar):
        ubar = np.ascontiguousarray(ubar, dtype=np.float64)
        a = np.zeros(2)
        rc = lib().oracle_max_wavespeed(C.byref(self.params), self.dim, self.ncell, _ptr(ubar),
                                        _ptr(a))
        if rc == ERR_NONPHYSICAL:
            raise NonPhysicalState("non-physical cell average")
        return a[: self.dim].copy()

    def rhs(self, ubar, mom, alpha):
        """Semi-discrete right-hand sides and the moment modifications.

        Returns (F1, Fmom, mom_hat) with F1 shaped like ubar and Fmom, mom_hat
        shaped like mom."""
        ubar = np.ascontiguousarray(ubar, dtype=np.float64)
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        F1 = np.empty_like(ubar)
        Fm = np.empty_like(mom)
        mh = np.empty_like(mom)
        if self.dim == 1:
            rc = lib().oracle_rhs_1d(C.byref(self.params), self.nx, self.dx, self.bc[0],
                                     self.bc[1], float(alpha[0]), _ptr(ubar),
                                     _ptr(np.ascontiguousarray(mom[0])), _ptr(F1),
                                     _ptr(Fm[0]), _ptr(mh[0]))
        else:
            bc = (C.c_int * 4)(*self.bc)
            al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
            v = np.ascontiguousarray(mom[0])
            w = np.ascontiguousarray(mom[1])
            rc = lib().oracle_rhs_2d(C.byref(self.params), self.nx, self.ny, self.dx, self.dy, bc,
                                     _ptr(al), _ptr(ubar), _ptr(v), _ptr(w), _ptr(F1),
                                     _ptr(Fm[0]), _ptr(Fm[1]), _ptr(mh[0]), _ptr(mh[1]))
        if rc == ERR_NONPHYSICAL:
            raise NonPhysicalState("non-physical cell average in the reconstruction")
        return F1, Fm, mh

    def stage(self, s, dt, alpha, ubar, mom, base=None):
        """One modified SSP-RK3 stage.  base = (u^n, v^n_hat) from stage 0.

        Returns (ubar_out, mom_out, base_out) where base_out is the stage-0
        base (u^n, v^n_hat) for s == 0 and `base` otherwise."""
        F1, Fm, mh = self.rhs(ubar, mom, alpha)
        u_new = ubar + dt * F1
        m_new = mh + dt * Fm
        if s == 0:
            return u_new, m_new, (np.array(ubar, dtype=np.float64, copy=True), mh)
        a, b = ((0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))[s - 1]
        return a * base[0] + b * u_new, a * base[1] + b * m_new, base

    def eigvecs(self, U, direction=0):
        """(R, L): the right eigenvectors (columns) the reconstruction
        projects with at the conserved state U, and L = R^-1 (Euler)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        n = self.dim + 2
        R = np.zeros(n * n)
        Linv = np.zeros(n * n)
        rc = lib().oracle_eigvecs(C.byref(self.params), _ptr(U), self.dim, int(direction),
                                  _ptr(R), _ptr(Linv))
        if rc == ERR_NONPHYSICAL:
            raise NonPhysicalState("non-physical state")
        return R.reshape(n, n), Linv.reshape(n, n)

    def roe_state(self, UL, UR):
        """The conserved state at the Roe average of UL and UR (Euler) that
        the per-interface projection takes its eigenvectors from."""
        UL = np.ascontiguousarray(UL, dtype=np.float64)
        UR = np.ascontiguousarray(UR, dtype=np.float64)
        U = np.zeros(self.dim + 2)
        rc = lib().oracle_roe_state(C.byref(self.params), _ptr(UL), _ptr(UR), self.dim,
                                    _ptr(U))
        if rc == ERR_NONPHYSICAL:
            raise NonPhysicalState("non-physical state")
        return U

    def check_physical(self, ubar):
        ubar = np.ascontiguousarray(ubar, dtype=np.float64)
        return bool(lib().oracle_all_physical(C.byref(self.params), self.dim, self.ncell,
                                              _ptr(ubar)))

    def step(self, ubar, mom, dt, alpha):
        u, m, base = self.stage(0, dt, alpha, ubar, mom)
        u, m, _ = self.stage(1, dt, alpha, u, m, base)
        u, m, _ = self.stage(2, dt, alpha, u, m, base)
        if self.eq == "euler" and not self.check_physical(u):
            raise NonPhysicalState("non-physical cell average after a step")
        return u, m

    def dt_from(self, alpha, cfl, h_power=1.0):
        """dt = CFL h^p / alpha in 1D, CFL / sum_d(alpha_d / h_d^p) in 2D."""
        if self.dim == 1:
            return cfl * self.dx ** h_power / alpha[0]
        return cfl / (alpha[0] / self.dx ** h_power + alpha[1] / self.dy ** h_power)

    def advance(self, ubar, mom, cfl=0.6, t_final=None, max_steps=None, h_power=1.0,
                fixed_dt=None, alpha=None):
        """Advance to t_final (or max_steps).  alpha: fixed LF coefficient, or
        None to take the maximum wave speed of U^n at every step."""
        t = 0.0
        steps = 0
        u, m = np.array(ubar, dtype=np.float64), np.array(mom, dtype=np.float64)
        while True:
            if max_steps is not None and steps >= max_steps:
                break
            if t_final is not None and t >= t_final * (1.0 - 1e-14):
                break
            a = np.asarray(alpha, dtype=np.float64) if alpha is not None else self.max_wavespeed(u)
            dt = fixed_dt if fixed_dt is not None else self.dt_from(a, cfl, h_power)
            if t_final is not None and t + dt > t_final:
                dt = t_final - t
            u, m = self.step(u, m, dt, a)
            t += dt
            steps += 1
        return u, m, t, steps
