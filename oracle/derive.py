"""Exact-rational derivation of the HWENO-U reconstruction operators.

TEST INFRASTRUCTURE ONLY.  This module is part of the CPU oracle: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The GPU library never reads anything produced here.

Everything is derived from the definitions in Section 2 of the paper, using
``fractions.Fraction`` and a plain Gauss-Jordan elimination, so that the
results are exact rationals:

* 1D quartic p0 (Section 2.1, Step 1): five moment conditions on the stencil
  {I_{i-1}, I_i, I_{i+1}} -- cell averages of the three cells and first-order
  moments of the two outer cells.  Linear p1, p2 from the averages of
  {I_{i-1}, I_i} and {I_i, I_{i+1}}.
* 2D quartic p0 (Section 2.2, Step 1): exact on the nine averages and on
  v4, v6, w2, w8, least squares on v2, v8, w4, w6 (constrained least
  squares, solved through its KKT system).  Linear p1..p4 from three averages
  each (stencils S1..S4 of the paper's Fig. 2.1).
* Smoothness indicators (Eq. (2.9) in 1D, Eq. (2.20) in 2D) as Gram matrices
  of the derivative integrals, in the normalised coordinates xi, eta.
* q-functionals: first-order moments of a polynomial over the target cell
  (the HWENO moment modification, Eq. (2.12) and (2.23)).

Coordinates: xi = (x - x_i)/dx, eta = (y - y_j)/dy; the target cell is
[-1/2, 1/2] (x [-1/2, 1/2]); neighbour k sits at offset k.

2D stencil labels follow the paper: label = 5 + a + 3 b for the cell at offset
(a, b), a, b in {-1, 0, 1}; so 1=(-1,-1), 2=(0,-1), 3=(1,-1), 4=(-1,0),
5=(0,0), 6=(1,0), 7=(-1,1), 8=(0,1), 9=(1,1).

2D monomial basis (the paper's phi_n ordering):
  1, xi, eta, xi^2, xi eta, eta^2, xi^3, xi^2 eta, xi eta^2, eta^3,
  xi^4, xi^3 eta, xi^2 eta^2, xi eta^3, eta^4.
"""
from fractions import Fraction as Fr
from functools import lru_cache

# ----------------------------------------------------------------------------
# small exact linear algebra
# ----------------------------------------------------------------------------


def solve(A, B):
    """Solve A X = B exactly (A square, B a list of rows, both Fractions)."""
    n = len(A)
    m = len(B[0])
    M = [list(A[r]) + list(B[r]) for r in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if M[r][col] != 0), None)
        if piv is None:
            raise ValueError("singular system")
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [v / p for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:n + m] for row in M]


def identity(n):
    return [[Fr(int(i == j)) for j in range(n)] for i in range(n)]


def matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def transpose(A):
    return [list(r) for r in zip(*A)]


# ----------------------------------------------------------------------------
# 1D
# ----------------------------------------------------------------------------


def seg_int(k, p):
    """Integral of xi^p over the cell at offset k, i.e. [k-1/2, k+1/2]."""
    lo, hi = Fr(2 * k - 1, 2), Fr(2 * k + 1, 2)
    return (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)


def mean_row_1d(k, deg):
    """Cell average of xi^l over cell k (length 1 in xi units), l = 0..deg."""
    return [seg_int(k, l) for l in range(deg + 1)]


def moment_row_1d(k, deg):
    """First-order moment (1/dx) int u (x-x_k)/dx dx of xi^l over cell k."""
    return [seg_int(k, l + 1) - k * seg_int(k, l) for l in range(deg + 1)]


@lru_cache(None)
def recon_1d():
    """Reconstruction operators in 1D.

    Returns a dict with
      'M0': 5x5, c0 = M0 @ [u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1}]
      'M1', 'M2': 2x5 (coefficients of the two linear polynomials, same data
              vector).
    """
    A = [mean_row_1d(-1, 4), mean_row_1d(0, 4), mean_row_1d(1, 4),
         moment_row_1d(-1, 4), moment_row_1d(1, 4)]
    M0 = solve(A, identity(5))
    # p1 on {I_{i-1}, I_i}: averages of cells -1, 0
    A1 = [mean_row_1d(-1, 1), mean_row_1d(0, 1)]
    X1 = solve(A1, identity(2))  # 2x2: coeffs from (u_{i-1}, u_i)
    M1 = [[X1[r][0], X1[r][1], Fr(0), Fr(0), Fr(0)] for r in range(2)]
    A2 = [mean_row_1d(0, 1), mean_row_1d(1, 1)]
    X2 = solve(A2, identity(2))  # from (u_i, u_{i+1})
    M2 = [[Fr(0), X2[r][0], X2[r][1], Fr(0), Fr(0)] for r in range(2)]
    return {"M0": M0, "M1": M1, "M2": M2}


def poly_deriv_1d(l, d):
    """d-th derivative of xi^l as (coefficient, power) or None."""
    if d > l:
        return None
    c = 1
    for t in range(d):
        c *= (l - t)
    return (c, l - d)


@lru_cache(None)
def beta_gram_1d(deg):
    """Gram matrix G with beta = c^T G c for p = sum c_l xi^l of degree deg.

    beta = sum_{l=1..deg} int_{I_i} dx^{2l-1} (d^l p/dx^l)^2 dx
         = sum_{l=1..deg} int_{-1/2}^{1/2} (d^l p/d xi^l)^2 d xi.
    """
    n = deg + 1
    G = [[Fr(0)] * n for _ in range(n)]
    for d in range(1, deg + 1):
        for a in range(n):
            da = poly_deriv_1d(a, d)
            if da is None:
                continue
            for b in range(n):
                db = poly_deriv_1d(b, d)
                if db is None:
                    continue
                G[a][b] += da[0] * db[0] * seg_int(0, da[1] + db[1])
    return G


def q_row_1d(deg):
    """q(p) = int_{-1/2}^{1/2} p(xi) xi d xi as a row over coefficients."""
    return [seg_int(0, l + 1) for l in range(deg + 1)]


# ----------------------------------------------------------------------------
# 2D
# ----------------------------------------------------------------------------

# the paper's phi_n ordering, as (power of xi, power of eta)
BASIS_2D = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1),
            (1, 2), (0, 3), (4, 0), (3, 1), (2, 2), (1, 3), (0, 4)]
BASIS_2D_LIN = BASIS_2D[:3]

# label -> offset (a, b)
OFFSETS_2D = {5 + a + 3 * b: (a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)}

# order of the 17 data values used by the 2D reconstruction
DATA_2D = ([("u", k) for k in range(1, 10)] + [("v", k) for k in (2, 4, 6, 8)]
           + [("w", k) for k in (2, 4, 6, 8)])


def _cell_row_2d(kind, label, basis):
    a, b = OFFSETS_2D[label]
    row = []
    for (p, q) in basis:
        if kind == "u":
            row.append(seg_int(a, p) * seg_int(b, q))
        elif kind == "v":
            row.append((seg_int(a, p + 1) - a * seg_int(a, p)) * seg_int(b, q))
        else:
            row.append(seg_int(a, p) * (seg_int(b, q + 1) - b * seg_int(b, q)))
    return row


@lru_cache(None)
def recon_2d():
    """Reconstruction operators in 2D.

    'M0' : 15x17, c0 = M0 @ data, data ordered as DATA_2D.
    'Mm' : list of four 3x17 matrices for p1..p4 (coefficients of 1, xi, eta).

    p0 matches the nine averages and v4, v6, w2, w8 exactly, and v2, v8, w4,
    w6 in the least-squares sense (Section 2.2, Step 1).  Solved as the KKT
    system  [2 B^T B  E^T; E  0] [c; lam] = [2 B^T d; e].
    """
    exact = [("u", k) for k in range(1, 10)] + [("v", 4), ("v", 6), ("w", 2), ("w", 8)]
    lsq = [("v", 2), ("v", 8), ("w", 4), ("w", 6)]
    E = [_cell_row_2d(kind, lab, BASIS_2D) for kind, lab in exact]
    B = [_cell_row_2d(kind, lab, BASIS_2D) for kind, lab in lsq]
    n = 15
    ne = len(E)
    BtB = matmul(transpose(B), B)
    K = [[Fr(0)] * (n + ne) for _ in range(n + ne)]
    for i in range(n):
        for j in range(n):
            K[i][j] = 2 * BtB[i][j]
        for j in range(ne):
            K[i][n + j] = E[j][i]
    for i in range(ne):
        for j in range(n):
            K[n + i][j] = E[i][j]
    # right-hand side as a linear map of the 17 data values
    R = [[Fr(0)] * 17 for _ in range(n + ne)]
    col = {key: idx for idx, key in enumerate(DATA_2D)}
    for r, key in enumerate(lsq):
        for i in range(n):
            R[i][col[key]] += 2 * B[r][i]
    for r, key in enumerate(exact):
        R[n + r][col[key]] = Fr(1)
    X = solve(K, R)
    M0 = X[:n]
    stencils = {1: (2, 4, 5), 2: (2, 5, 6), 3: (4, 5, 8), 4: (5, 6, 8)}
    Mm = []
    for m in (1, 2, 3, 4):
        labs = stencils[m]
        A = [_cell_row_2d("u", lab, BASIS_2D_LIN) for lab in labs]
        Xm = solve(A, identity(3))
        Mfull = [[Fr(0)] * 17 for _ in range(3)]
        for r in range(3):
            for t, lab in enumerate(labs):
                Mfull[r][col[("u", lab)]] = Xm[r][t]
        Mm.append(Mfull)
    return {"M0": M0, "Mm": Mm}


def _mono_deriv(pq, d):
    """Derivative d=(d1,d2) of xi^p eta^q: (coefficient, (p', q')) or None."""
    (p, q), (d1, d2) = pq, d
    if d1 > p or d2 > q:
        return None
    c = 1
    for t in range(d1):
        c *= (p - t)
    for t in range(d2):
        c *= (q - t)
    return (c, (p - d1, q - d2))


@lru_cache(None)
def beta_gram_2d(deg):
    """Gram matrix of the 2D smoothness indicator for a degree-deg polynomial.

    beta = sum_{1<=|l|<=deg} |I|^{|l|-1} int_I (D^l p)^2 dx dy, which for
    dx = dy reduces to the same sum of integrals over [-1/2,1/2]^2 in the
    normalised variables; every multi-index l = (l1, l2) is counted once.
    """
    basis = [b for b in BASIS_2D if b[0] + b[1] <= deg]
    n = len(basis)
    G = [[Fr(0)] * n for _ in range(n)]
    for order in range(1, deg + 1):
        for d1 in range(order + 1):
            d = (d1, order - d1)
            for a in range(n):
                da = _mono_deriv(basis[a], d)
                if da is None:
                    continue
                for b in range(n):
                    db = _mono_deriv(basis[b], d)
                    if db is None:
                        continue
                    pa, pb = da[1], db[1]
                    G[a][b] += (da[0] * db[0] * seg_int(0, pa[0] + pb[0])
                                * seg_int(0, pa[1] + pb[1]))
    return G


def q_rows_2d(deg):
    """(q^v, q^w) rows: int p xi and int p eta over the target cell."""
    basis = [b for b in BASIS_2D if b[0] + b[1] <= deg]
    qv = [seg_int(0, p + 1) * seg_int(0, q) for (p, q) in basis]
    qw = [seg_int(0, p) * seg_int(0, q + 1) for (p, q) in basis]
    return qv, qw


def as_float_rows(M):
    return [[float(v) for v in row] for row in M]
