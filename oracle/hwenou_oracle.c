/*
 * HWENO-U CPU oracle (FP64).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load.  It shares no code, header, table or constant generator with the GPU
 * library.  The reconstruction operators (the 1D 5x5 and 2D 15x17 matrices,
 * the smoothness-indicator Gram matrices and the moment functionals) are
 * derived exactly from the moment conditions by oracle/derive.py and handed
 * in through oracle_set_ops_1d / oracle_set_ops_2d.
 *
 * It follows the steps of Section 2 of Fan, Qiu & Zhao, "A moment-based
 * Hermite WENO scheme with unified stencils for hyperbolic conservation
 * laws", cell by cell, with plain loops:
 *   Step 1  polynomials p0 (quartic) and p_m (linear)         -- Sec. 2.1 / 2.2
 *   Step 2  smoothness indicators beta_m = c^T G c            -- Eq. (2.9)/(2.20)
 *   Step 3  tau, u_ave, scale-invariant nonlinear weights     -- Eq. (2.10)-(2.11)/(2.21)-(2.22)
 *           reconstruction u_i(x) and moment modification v^ -- Eq. (2.12)/(2.23)
 *   semi-discrete right-hand sides with Lax-Friedrichs fluxes -- Eq. (2.3)-(2.4)/(2.16)
 * The Runge-Kutta combination (Eq. (2.13)) is done by the Python driver.
 * For the Euler equations the reconstruction runs on local characteristic
 * variables (Remark 2.2), projected with the eigenvectors of the flux
 * Jacobian at the target cell's average; in 2D an x-sweep (eigenvectors of
 * f') yields the x-edge values, the interior values used for f and v^, and a
 * y-sweep (eigenvectors of g') the y-edge values, the interior values used
 * for g and w^.  L = R^{-1} is obtained here by Gauss-Jordan elimination.
 * The remark leaves the state of the eigenvectors open; besides the cell's
 * own average (the default), a per-interface variant takes the edge values
 * at an interface in the characteristic variables of the Roe average of the
 * two cells that share it, as the classical characteristic WENO schemes do,
 * and keeps the cell's own average for the interior values and v^, w^.
 *
 * ORACLE_PLANT (test-only compile switch, never set in the library that the
 * tests and the benchmark load) plants one known mistake, so that the tests
 * can show that a pin fails on it: 1 = energy entry q^2 instead of q^2/2 in the
 * entropy eigenvector; 2 = the 2D tau averaged over 2 instead of the 4
 * differences; 3 = the 2D u_ave taken over all nine stencil cells; 4 = the
 * arithmetic mean of the two enthalpies in the Roe average; 5 = the edge
 * values of each side of a cell taken in the basis of the interface on the
 * other side (per-interface projection).
 */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Loops over fewer values than this run on one thread: every cell is
 * computed independently, so the results do not depend on the thread count,
 * and small grids stepped thousands of times would spend their time in the
 * start-up of parallel regions. */
#define ORACLE_OMP_MIN 16384
#define ORACLE_OMP_MIN_2D 256 /* cells: a 2D cell costs ~30 times a 1D value */

#define EQ_ADVECTION 0
#define EQ_BURGERS 1
#define EQ_EULER 2

#define W_SCALE_INVARIANT 0
#define W_ZQ 1
#define W_LINEAR 2

#define BC_PERIODIC 0
#define BC_TRANSMISSIVE 1
#define BC_REFLECTIVE 2

#define ERR_NONPHYSICAL 4

typedef struct {
  int eq;          /* EQ_* */
  int ncomp;       /* 1 for scalar laws; 3 (1D) or 4 (2D) for Euler */
  int weights;     /* W_* */
  int char_decomp; /* Euler: 0 = component-wise; 1 = characteristic-wise, the
                      x-sweep in x-characteristic variables, the y-sweep in
                      y-characteristic variables; 2 = characteristic-wise with
                      the single x-projection for every output (2D); 3 = as 1,
                      but the edge values at each interface in the
                      characteristic variables of the Roe average of the two
                      cells that share it (2D) */
  double adv_x, adv_y;   /* advection velocity */
  double gas_gamma;      /* ratio of specific heats */
  double gamma_low;      /* linear weight of each linear polynomial */
  double eps;            /* epsilon in the nonlinear weights */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* operators handed in from the exact derivation                            */
/* ------------------------------------------------------------------------ */
static double OP1_M0[5 * 5], OP1_M1[2 * 5], OP1_M2[2 * 5];
static double OP1_G0[5 * 5], OP1_G1[2 * 2];
static double OP1_Q0[5], OP1_Q1[2];

static double OP2_M0[15 * 17], OP2_MM[4 * 3 * 17];
static double OP2_G0[15 * 15], OP2_G1[3 * 3];
static double OP2_QV0[15], OP2_QW0[15], OP2_QV1[3], OP2_QW1[3];

void oracle_set_ops_1d(const double *M0, const double *M1, const double *M2,
                       const double *G0, const double *G1, const double *Q0,
                       const double *Q1) {
  memcpy(OP1_M0, M0, sizeof OP1_M0);
  memcpy(OP1_M1, M1, sizeof OP1_M1);
  memcpy(OP1_M2, M2, sizeof OP1_M2);
  memcpy(OP1_G0, G0, sizeof OP1_G0);
  memcpy(OP1_G1, G1, sizeof OP1_G1);
  memcpy(OP1_Q0, Q0, sizeof OP1_Q0);
  memcpy(OP1_Q1, Q1, sizeof OP1_Q1);
}

void oracle_set_ops_2d(const double *M0, const double *MM, const double *G0,
                       const double *G1, const double *QV0, const double *QW0,
                       const double *QV1, const double *QW1) {
  memcpy(OP2_M0, M0, sizeof OP2_M0);
  memcpy(OP2_MM, MM, sizeof OP2_MM);
  memcpy(OP2_G0, G0, sizeof OP2_G0);
  memcpy(OP2_G1, G1, sizeof OP2_G1);
  memcpy(OP2_QV0, QV0, sizeof OP2_QV0);
  memcpy(OP2_QW0, QW0, sizeof OP2_QW0);
  memcpy(OP2_QV1, QV1, sizeof OP2_QV1);
  memcpy(OP2_QW1, QW1, sizeof OP2_QW1);
}

/* ------------------------------------------------------------------------ */
/* helpers                                                                  */
/* ------------------------------------------------------------------------ */
/* Source cell of index i of a grid of n cells (|overshoot| <= 2):
 * periodic wrap, transmissive copy of the boundary cell, or reflective
 * mirror image (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2).  *mirror is set
 * to 1 for a mirror image. */
static int bc_index(int i, int n, int bc_lo, int bc_hi, int *mirror) {
  *mirror = 0;
  if (i < 0) {
    if (bc_lo == BC_PERIODIC) return ((i % n) + n) % n;
    if (bc_lo == BC_REFLECTIVE) { *mirror = 1; return -1 - i; }
    return 0;
  }
  if (i >= n) {
    if (bc_hi == BC_PERIODIC) return i % n;
    if (bc_hi == BC_REFLECTIVE) { *mirror = 1; return 2 * n - 1 - i; }
    return n - 1;
  }
  return i;
}

/* Euler data of a cell mirrored across a wall normal to direction d: the
 * normal momentum (component 1 + d) changes sign, and a moment along d
 * changes sign once more because its local coordinate does.  e is the
 * moment direction, or -1 for the cell average. */
static double mirror_sign(int k, int d, int e) {
  const double s = k == 1 + d ? -1.0 : 1.0;
  return e == d ? -s : s;
}

static double quad_form(const double *G, const double *c, int n) {
  double s = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) s += c[a] * G[a * n + b] * c[b];
  return s;
}

static double dot(const double *a, const double *b, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

static void matvec(const double *M, const double *x, double *y, int rows, int cols) {
  for (int r = 0; r < rows; ++r) y[r] = dot(M + r * cols, x, cols);
}

/* Nonlinear weights of Step 3.  beta[0..nm], nm linear polynomials.
 * tau = (mean_m |beta_0 - beta_m|)^2, w~_m = g_m (1 + tau/(beta_m u_ave + eps)). */
static void nonlinear_weights(const oracle_params *P, const double *beta, int nm,
                              double u_ave, const double *lin, double *w) {
  if (P->weights == W_LINEAR) {
    for (int m = 0; m <= nm; ++m) w[m] = lin[m];
    return;
  }
  if (P->weights == W_ZQ) u_ave = 1.0;
  double t = 0.0;
  for (int m = 1; m <= nm; ++m) t += fabs(beta[0] - beta[m]);
  t /= (ORACLE_PLANT == 2 && nm == 4) ? 2 : nm;
  double tau = t * t;
  double sum = 0.0;
  for (int m = 0; m <= nm; ++m) {
    w[m] = lin[m] * (1.0 + tau / (beta[m] * u_ave + P->eps));
    sum += w[m];
  }
  for (int m = 0; m <= nm; ++m) w[m] /= sum;
}

/* ------------------------------------------------------------------------ */
/* 1D scalar HWENO reconstruction of one cell                               */
/* ------------------------------------------------------------------------ */
static double gl4_nodes[4]; /* filled in oracle_rhs_1d: -1/2, -sqrt(5)/10, sqrt(5)/10, 1/2 */
static const double GL4_W[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};

static double poly1d(const double *c, int deg, double xi) {
  double s = 0.0, p = 1.0;
  for (int l = 0; l <= deg; ++l) {
    s += c[l] * p;
    p *= xi;
  }
  return s;
}

/* s = (u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1}); out: values at the four
 * Gauss-Lobatto nodes and the modified moment v^. */
static void recon_1d_scalar(const oracle_params *P, const double s[5], double pts[4],
                            double *vhat) {
  double c0[5], c1[2], c2[2];
  matvec(OP1_M0, s, c0, 5, 5);
  matvec(OP1_M1, s, c1, 2, 5);
  matvec(OP1_M2, s, c2, 2, 5);
  double beta[3] = {quad_form(OP1_G0, c0, 5), quad_form(OP1_G1, c1, 2),
                    quad_form(OP1_G1, c2, 2)};
  double ua = (fabs(s[0]) + fabs(s[1]) + fabs(s[2])) / 3.0;
  double u_ave = ua * ua;
  double g0 = 1.0 - 2.0 * P->gamma_low;
  double lin[3] = {g0, P->gamma_low, P->gamma_low};
  double w[3];
  nonlinear_weights(P, beta, 2, u_ave, lin, w);
  for (int G = 0; G < 4; ++G) {
    double xi = gl4_nodes[G];
    double p0 = poly1d(c0, 4, xi), p1 = poly1d(c1, 1, xi), p2 = poly1d(c2, 1, xi);
    pts[G] = w[0] * (p0 / g0 - lin[1] / g0 * p1 - lin[2] / g0 * p2) + w[1] * p1 + w[2] * p2;
  }
  double q0 = dot(OP1_Q0, c0, 5), q1 = dot(OP1_Q1, c1, 2), q2 = dot(OP1_Q1, c2, 2);
  *vhat = w[0] * (q0 / g0 - lin[1] / g0 * q1 - lin[2] / g0 * q2) + w[1] * q1 + w[2] * q2;
}

/* ------------------------------------------------------------------------ */
/* Euler eigenvectors                                                       */
/* ------------------------------------------------------------------------ */
/* Inverse of an n x n matrix by Gauss-Jordan with partial pivoting. */
static int invert(const double *A, double *Ainv, int n) {
  double M[4][8];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) M[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (M[piv][col] == 0.0 || !isfinite(M[piv][col])) return -1;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = M[col][c];
        M[col][c] = M[piv][c];
        M[piv][c] = t;
      }
    double p = M[col][col];
    for (int c = 0; c < 2 * n; ++c) M[col][c] /= p;
    for (int r = 0; r < n; ++r)
      if (r != col) {
        double f = M[r][col];
        for (int c = 0; c < 2 * n; ++c) M[r][c] -= f * M[col][c];
      }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ainv[r * n + c] = M[r][c + n];
  return 0;
}

/* Right eigenvectors (columns) of the Euler flux Jacobian in direction dir
 * (0 = x, 1 = y) at the conserved state U.  Returns -1 on a nonphysical
 * state.  1D: columns (1, u-c, H-uc), (1, u, u^2/2), (1, u+c, H+uc).
 * 2D, x: (1,u-c,v,H-uc), (1,u,v,q^2/2), (0,0,1,v), (1,u+c,v,H+uc);
 * 2D, y: (1,u,v-c,H-vc), (1,u,v,q^2/2), (0,1,0,u), (1,u,v+c,H+vc). */
static int euler_right_eigvecs(const oracle_params *P, const double *U, int dim, int dir,
                               double *R) {
  double gm = P->gas_gamma;
  double rho = U[0];
  if (!(rho > 0.0)) return -1;
  double u = U[1] / rho;
  double v = dim == 2 ? U[2] / rho : 0.0;
  double E = U[dim + 1];
  double q2 = u * u + v * v;
  double p = (gm - 1.0) * (E - 0.5 * rho * q2);
  if (!(p > 0.0)) return -1;
  double c = sqrt(gm * p / rho);
  double H = (E + p) / rho;
  if (dim == 1) {
    const double e1 = ORACLE_PLANT == 1 ? u * u : 0.5 * u * u;
    double cols[3][3] = {{1.0, u - c, H - u * c}, {1.0, u, e1}, {1.0, u + c, H + u * c}};
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) R[r * 3 + k] = cols[k][r];
  } else if (dir == 0) {
    const double e1 = ORACLE_PLANT == 1 ? q2 : 0.5 * q2;
    double cols[4][4] = {{1.0, u - c, v, H - u * c},
                         {1.0, u, v, e1},
                         {0.0, 0.0, 1.0, v},
                         {1.0, u + c, v, H + u * c}};
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k) R[r * 4 + k] = cols[k][r];
  } else {
    const double e1 = ORACLE_PLANT == 1 ? q2 : 0.5 * q2;
    double cols[4][4] = {{1.0, u, v - c, H - v * c},
                         {1.0, u, v, e1},
                         {0.0, 1.0, 0.0, u},
                         {1.0, u, v + c, H + v * c}};
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k) R[r * 4 + k] = cols[k][r];
  }
  return 0;
}

/* Roe average of two conserved states (ideal gas): sqrt(rho)-weighted
 * velocity and total enthalpy, returned as a conserved state with density
 * sqrt(rho_L rho_R) and the energy that gives that enthalpy, so that
 * euler_right_eigvecs sees u, v, H and c^2 = (gamma - 1)(H - q^2/2).
 * Returns -1 on a non-physical input. */
static int roe_state(const oracle_params *P, const double *UL, const double *UR, int dim,
                     double *U) {
  double gm = P->gas_gamma;
  if (!(UL[0] > 0.0) || !(UR[0] > 0.0)) return -1;
  double sl = sqrt(UL[0]), sr = sqrt(UR[0]);
  double w = 1.0 / (sl + sr);
  double q2 = 0.0, vel[2];
  for (int d = 0; d < dim; ++d) {
    vel[d] = (UL[1 + d] / sl + UR[1 + d] / sr) * w; /* (sl u_L + sr u_R)/(sl + sr) */
    q2 += vel[d] * vel[d];
  }
  double hl = 0.0, hr = 0.0, ql = 0.0, qr = 0.0;
  for (int d = 0; d < dim; ++d) {
    ql += UL[1 + d] * UL[1 + d];
    qr += UR[1 + d] * UR[1 + d];
  }
  double pl = (gm - 1.0) * (UL[dim + 1] - 0.5 * ql / UL[0]);
  double pr = (gm - 1.0) * (UR[dim + 1] - 0.5 * qr / UR[0]);
  if (!(pl > 0.0) || !(pr > 0.0)) return -1;
  hl = (UL[dim + 1] + pl) / UL[0];
  hr = (UR[dim + 1] + pr) / UR[0];
  double H = ORACLE_PLANT == 4 ? 0.5 * (hl + hr) : (sl * hl + sr * hr) * w;
  double rho = sl * sr;
  U[0] = rho;
  for (int d = 0; d < dim; ++d) U[1 + d] = rho * vel[d];
  U[dim + 1] = (rho * H + (gm - 1.0) * 0.5 * rho * q2) / gm;
  return 0;
}

int oracle_roe_state(const oracle_params *P, const double *UL, const double *UR, int dim,
                     double *U) {
  return roe_state(P, UL, UR, dim, U) ? ERR_NONPHYSICAL : 0;
}

/* The eigenvector basis the reconstruction projects with, for the tests:
 * R (right eigenvectors as columns, row-major n x n) and L = R^{-1}, at the
 * conserved state U (n = dim + 2).  Returns 0, or ERR_NONPHYSICAL. */
int oracle_eigvecs(const oracle_params *P, const double *U, int dim, int dir, double *R,
                   double *L) {
  if (euler_right_eigvecs(P, U, dim, dir, R) || invert(R, L, dim + 2)) return ERR_NONPHYSICAL;
  return 0;
}

/* physical fluxes: dir 0 = f (x), dir 1 = g (y) */
static void phys_flux(const oracle_params *P, int dim, int dir, const double *U, double *F) {
  if (P->eq == EQ_ADVECTION) {
    F[0] = (dir == 0 ? P->adv_x : P->adv_y) * U[0];
    return;
  }
  if (P->eq == EQ_BURGERS) {
    F[0] = 0.5 * U[0] * U[0];
    return;
  }
  double gm = P->gas_gamma;
  double rho = U[0];
  if (dim == 1) {
    double u = U[1] / rho;
    double p = (gm - 1.0) * (U[2] - 0.5 * rho * u * u);
    F[0] = U[1];
    F[1] = U[1] * u + p;
    F[2] = u * (U[2] + p);
    return;
  }
  double u = U[1] / rho, v = U[2] / rho;
  double p = (gm - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
  if (dir == 0) {
    F[0] = U[1];
    F[1] = U[1] * u + p;
    F[2] = U[2] * u;
    F[3] = u * (U[3] + p);
  } else {
    F[0] = U[2];
    F[1] = U[1] * v;
    F[2] = U[2] * v + p;
    F[3] = v * (U[3] + p);
  }
}

static int is_physical(const oracle_params *P, int dim, const double *U) {
  for (int k = 0; k < P->ncomp; ++k)
    if (!isfinite(U[k])) return 0;
  if (P->eq != EQ_EULER) return 1;
  double rho = U[0];
  if (!(rho > 0.0)) return 0;
  double q2 = 0.0;
  for (int d = 0; d < dim; ++d) q2 += U[1 + d] * U[1 + d];
  double p = (P->gas_gamma - 1.0) * (U[dim + 1] - 0.5 * q2 / rho);
  return p > 0.0;
}

/* ------------------------------------------------------------------------ */
/* 1D right-hand side                                                       */
/* ------------------------------------------------------------------------ */
/* ubar, vbar: [ncomp][n].  alpha: LF coefficient.  Outputs F1, F2, vhat:
 * [ncomp][n].  Returns 0, or ERR_NONPHYSICAL. */
int oracle_rhs_1d(const oracle_params *P, int n, double dx, int bc_lo, int bc_hi, double alpha,
                  const double *ubar, const double *vbar, double *F1, double *F2,
                  double *vhat) {
  const int nc = P->ncomp;
  gl4_nodes[0] = -0.5;
  gl4_nodes[1] = -sqrt(5.0) / 10.0;
  gl4_nodes[2] = sqrt(5.0) / 10.0;
  gl4_nodes[3] = 0.5;
  const int ne = n + 2; /* cells -1 .. n */
  double *pts = (double *)malloc(sizeof(double) * (size_t)ne * 4 * nc);
  double *vh = (double *)malloc(sizeof(double) * (size_t)ne * nc);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) if (ne * nc >= ORACLE_OMP_MIN)
  for (int e = 0; e < ne; ++e) {
    int i = e - 1;
    int idx[3], mir[3];
    for (int d = -1; d <= 1; ++d) idx[d + 1] = bc_index(i + d, n, bc_lo, bc_hi, mir + d + 1);
    /* sign of the average / moment of stencil cell t, component k */
#define SU1(t, k) (mir[t] ? mirror_sign(k, 0, -1) : 1.0)
#define SV1(t, k) (mir[t] ? mirror_sign(k, 0, 0) : 1.0)
    double *cp = pts + (size_t)e * 4 * nc;
    double *cv = vh + (size_t)e * nc;
    if (P->eq != EQ_EULER || !P->char_decomp) {
      for (int k = 0; k < nc; ++k) {
        const double *u = ubar + (size_t)k * n, *v = vbar + (size_t)k * n;
        double s[5] = {SU1(0, k) * u[idx[0]], SU1(1, k) * u[idx[1]], SU1(2, k) * u[idx[2]],
                       SV1(0, k) * v[idx[0]], SV1(2, k) * v[idx[2]]};
        double p4[4];
        recon_1d_scalar(P, s, p4, cv + k);
        for (int G = 0; G < 4; ++G) cp[G * nc + k] = p4[G];
      }
      continue;
    }
    /* characteristic-wise: project the five stencil vectors with L(u_i) */
    double Ui[3], R[9], L[9];
    for (int k = 0; k < 3; ++k) Ui[k] = SU1(1, k) * ubar[(size_t)k * n + idx[1]];
    if (euler_right_eigvecs(P, Ui, 1, 0, R) || invert(R, L, 3)) {
      bad |= 1;
      continue;
    }
    double S[5][3];
    for (int k = 0; k < 3; ++k) {
      const double *u = ubar + (size_t)k * n, *v = vbar + (size_t)k * n;
      S[0][k] = SU1(0, k) * u[idx[0]];
      S[1][k] = SU1(1, k) * u[idx[1]];
      S[2][k] = SU1(2, k) * u[idx[2]];
      S[3][k] = SV1(0, k) * v[idx[0]];
      S[4][k] = SV1(2, k) * v[idx[2]];
    }
#undef SU1
#undef SV1
    double Wp[4][3], Wv[3];
    for (int ch = 0; ch < 3; ++ch) {
      double s[5];
      for (int t = 0; t < 5; ++t) s[t] = dot(L + ch * 3, S[t], 3);
      double p4[4];
      recon_1d_scalar(P, s, p4, Wv + ch);
      for (int G = 0; G < 4; ++G) Wp[G][ch] = p4[G];
    }
    for (int G = 0; G < 4; ++G) matvec(R, Wp[G], cp + G * nc, 3, 3);
    matvec(R, Wv, cv, 3, 3);
  }
  if (bad) {
    free(pts);
    free(vh);
    return ERR_NONPHYSICAL;
  }
  /* interface fluxes fh[e] at x_{i+1/2}, i = e-1, e = 0..n */
  double *fh = (double *)malloc(sizeof(double) * (size_t)(n + 1) * nc);
#pragma omp parallel for schedule(static) if (n * nc >= ORACLE_OMP_MIN)
  for (int e = 0; e <= n; ++e) {
    const double *um = pts + (size_t)e * 4 * nc + 3 * nc;      /* cell e-1 at +1/2 */
    const double *up = pts + (size_t)(e + 1) * 4 * nc + 0 * nc; /* cell e at -1/2 */
    double fm[4], fp[4];
    phys_flux(P, 1, 0, um, fm);
    phys_flux(P, 1, 0, up, fp);
    for (int k = 0; k < nc; ++k)
      fh[(size_t)e * nc + k] = 0.5 * (fm[k] + fp[k] - alpha * (up[k] - um[k]));
  }
#pragma omp parallel for schedule(static) if (n * nc >= ORACLE_OMP_MIN)
  for (int i = 0; i < n; ++i) {
    const double *fl = fh + (size_t)i * nc;       /* x_{i-1/2} */
    const double *fr = fh + (size_t)(i + 1) * nc; /* x_{i+1/2} */
    const double *cp = pts + (size_t)(i + 1) * 4 * nc;
    double vol[4] = {0, 0, 0, 0};
    for (int G = 0; G < 4; ++G) {
      double f[4];
      phys_flux(P, 1, 0, cp + G * nc, f);
      for (int k = 0; k < nc; ++k) vol[k] += GL4_W[G] * f[k];
    }
    for (int k = 0; k < nc; ++k) {
      F1[(size_t)k * n + i] = -(fr[k] - fl[k]) / dx;
      F2[(size_t)k * n + i] = -(fl[k] + fr[k]) / (2.0 * dx) + vol[k] / dx;
      vhat[(size_t)k * n + i] = vh[(size_t)(i + 1) * nc + k];
    }
  }
  free(fh);
  free(pts);
  free(vh);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* 2D scalar HWENO reconstruction of one cell                               */
/* ------------------------------------------------------------------------ */
static const int B2P[15] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
static const int B2Q[15] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};

static double ipow(double x, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= x;
  return r;
}

/* phi_n at the 21 output points, filled once per call of oracle_rhs_2d */
static double PHI2[21][15];

static double poly2d_at(const double *c, int nb, int Pt) {
  double s = 0.0;
  for (int n = 0; n < nb; ++n) s += c[n] * PHI2[Pt][n];
  return s;
}

static double g3_nodes[3];
static const double G3_W[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};

/* Output points of one reconstruction, index layout:
 *   x-edges  (xi = -1/2, eta_G) at 0..2, (xi = +1/2, eta_G) at 3..5
 *   y-edges  (xi_G, eta = -1/2) at 6..8, (xi_G, eta = +1/2) at 9..11
 *   interior (xi_G, eta_H) at 12 + 3*G + H                               */
#define NPTS2 21
static void point_coords_2d(int P, double *xi, double *eta) {
  if (P < 6) {
    *xi = P < 3 ? -0.5 : 0.5;
    *eta = g3_nodes[P % 3];
  } else if (P < 12) {
    *xi = g3_nodes[(P - 6) % 3];
    *eta = P < 9 ? -0.5 : 0.5;
  } else {
    *xi = g3_nodes[(P - 12) / 3];
    *eta = g3_nodes[(P - 12) % 3];
  }
}

/* d = 17 data values (DATA_2D order: u1..u9, v2, v4, v6, v8, w2, w4, w6, w8).
 * Writes all 21 point values and (v^, w^). */
static void recon_2d_scalar(const oracle_params *P, const double d[17], double pts[NPTS2],
                            double *vhat, double *what) {
  double c0[15], cm[4][3];
  matvec(OP2_M0, d, c0, 15, 17);
  for (int m = 0; m < 4; ++m) matvec(OP2_MM + m * 3 * 17, d, cm[m], 3, 17);
  double beta[5];
  beta[0] = quad_form(OP2_G0, c0, 15);
  for (int m = 0; m < 4; ++m) beta[m + 1] = quad_form(OP2_G1, cm[m], 3);
  /* u_ave over cells 2, 4, 5, 6, 8 */
  double ua = (fabs(d[1]) + fabs(d[3]) + fabs(d[4]) + fabs(d[5]) + fabs(d[7])) / 5.0;
  if (ORACLE_PLANT == 3) {
    ua = 0.0;
    for (int t = 0; t < 9; ++t) ua += fabs(d[t]);
    ua /= 9.0;
  }
  double u_ave = ua * ua;
  double g0 = 1.0 - 4.0 * P->gamma_low;
  double lin[5] = {g0, P->gamma_low, P->gamma_low, P->gamma_low, P->gamma_low};
  double w[5];
  nonlinear_weights(P, beta, 4, u_ave, lin, w);
  for (int Pt = 0; Pt < NPTS2; ++Pt) {
    double p0 = poly2d_at(c0, 15, Pt);
    double inner = p0 / g0, outer = 0.0;
    for (int m = 0; m < 4; ++m) {
      double pm = poly2d_at(cm[m], 3, Pt);
      inner -= lin[m + 1] / g0 * pm;
      outer += w[m + 1] * pm;
    }
    pts[Pt] = w[0] * inner + outer;
  }
  double qv_in = dot(OP2_QV0, c0, 15) / g0, qw_in = dot(OP2_QW0, c0, 15) / g0;
  double qv_out = 0.0, qw_out = 0.0;
  for (int m = 0; m < 4; ++m) {
    double qv = dot(OP2_QV1, cm[m], 3), qw = dot(OP2_QW1, cm[m], 3);
    qv_in -= lin[m + 1] / g0 * qv;
    qw_in -= lin[m + 1] / g0 * qw;
    qv_out += w[m + 1] * qv;
    qw_out += w[m + 1] * qw;
  }
  *vhat = w[0] * qv_in + qv_out;
  *what = w[0] * qw_in + qw_out;
}

/* Component-wise reconstruction of the 17 stencil vectors D[t][k]. */
static void recon_components_2d(const oracle_params *P, double D[17][4], int nc,
                                double pts[NPTS2][4], double *vh, double *wh) {
  for (int ch = 0; ch < nc; ++ch) {
    double d[17], p[NPTS2];
    for (int t = 0; t < 17; ++t) d[t] = D[t][ch];
    recon_2d_scalar(P, d, p, vh + ch, wh + ch);
    for (int Pt = 0; Pt < NPTS2; ++Pt) pts[Pt][ch] = p[Pt];
  }
}

/* Characteristic reconstruction of the 17 stencil vectors D[t][k] with the
 * eigenvectors of the flux Jacobian in direction `sweep` at the state Uref:
 * project with L = R^-1, reconstruct each field, map the point values and
 * moments back with R.  Returns -1 on a non-physical Uref. */
static int project_recon_2d(const oracle_params *P, double D[17][4], const double *Uref,
                            int sweep, int nc, double pts[NPTS2][4], double *vh, double *wh) {
  double R[16], L[16];
  if (euler_right_eigvecs(P, Uref, 2, sweep, R) || invert(R, L, 4)) return -1;
  double W[NPTS2][4], Wv[4], Ww[4];
  for (int ch = 0; ch < nc; ++ch) {
    double d[17], p[NPTS2];
    for (int t = 0; t < 17; ++t) d[t] = dot(L + ch * 4, D[t], 4);
    recon_2d_scalar(P, d, p, Wv + ch, Ww + ch);
    for (int Pt = 0; Pt < NPTS2; ++Pt) W[Pt][ch] = p[Pt];
  }
  for (int Pt = 0; Pt < NPTS2; ++Pt) matvec(R, W[Pt], pts[Pt], 4, 4);
  matvec(R, Wv, vh, 4, 4);
  matvec(R, Ww, wh, 4, 4);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* 2D right-hand side                                                       */
/* ------------------------------------------------------------------------ */
/* Per extended cell (nx+2)(ny+2) storage of the sweep outputs. */
typedef struct {
  double xe[6][4];  /* x-edge values (x-sweep)           */
  double ye[6][4];  /* y-edge values (y-sweep)           */
  double volf[4];   /* sum_G sum_H w_G w_H f(u(xi_G, eta_H)) (x-sweep) */
  double volg[4];   /* same with g (y-sweep)                           */
  double vh[4], wh[4];
} cell2d;

/* ubar, vbar, wbar: [ncomp][ny][nx].  alpha[2] = (alpha_1, alpha_2).
 * bc[4] = (x-lo, x-hi, y-lo, y-hi).  Outputs F1, F2, F3, vhat, what with
 * the same layout.  Returns 0 or ERR_NONPHYSICAL. */
int oracle_rhs_2d(const oracle_params *P, int nx, int ny, double dx, double dy, const int *bc,
                  const double *alpha, const double *ubar, const double *vbar,
                  const double *wbar, double *F1, double *F2, double *F3, double *vhat,
                  double *what) {
  const int nc = P->ncomp;
  const size_t plane = (size_t)nx * ny;
  g3_nodes[0] = -sqrt(15.0) / 10.0;
  g3_nodes[1] = 0.0;
  g3_nodes[2] = sqrt(15.0) / 10.0;
  for (int Pt = 0; Pt < NPTS2; ++Pt) {
    double xi, eta;
    point_coords_2d(Pt, &xi, &eta);
    for (int n = 0; n < 15; ++n) PHI2[Pt][n] = ipow(xi, B2P[n]) * ipow(eta, B2Q[n]);
  }
  const int ex = nx + 2, ey = ny + 2;
  cell2d *C = (cell2d *)calloc((size_t)ex * ey, sizeof(cell2d));
  int bad = 0;
  /* labels 1..9 -> offsets (a, b): label = 5 + a + 3 b */
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad) if (ex * ey >= ORACLE_OMP_MIN_2D)
  for (int ej = 0; ej < ey; ++ej) {
    for (int ei = 0; ei < ex; ++ei) {
      int i = ei - 1, j = ej - 1;
      /* corner cells of the extended grid are never needed */
      if ((i < 0 || i >= nx) && (j < 0 || j >= ny)) continue;
      size_t at[10];
      int mx[10], my[10];
      for (int lab = 1; lab <= 9; ++lab) {
        int a = (lab - 1) % 3 - 1, b = (lab - 1) / 3 - 1;
        int ii = bc_index(i + a, nx, bc[0], bc[1], mx + lab);
        int jj = bc_index(j + b, ny, bc[2], bc[3], my + lab);
        at[lab] = (size_t)jj * nx + ii;
      }
      cell2d *out = C + (size_t)ej * ex + ei;
      /* gather data vectors per conserved component: DATA_2D order; mirror
       * images across x- and y-walls take the signs of mirror_sign() */
      double D[17][4];
      for (int k = 0; k < nc; ++k) {
        for (int lab = 1; lab <= 9; ++lab)
          D[lab - 1][k] = (mx[lab] ? mirror_sign(k, 0, -1) : 1.0) *
                          (my[lab] ? mirror_sign(k, 1, -1) : 1.0) * ubar[k * plane + at[lab]];
        const int ml[4] = {2, 4, 6, 8};
        for (int t = 0; t < 4; ++t) {
          const int lab = ml[t];
          D[9 + t][k] = (mx[lab] ? mirror_sign(k, 0, 0) : 1.0) *
                        (my[lab] ? mirror_sign(k, 1, 0) : 1.0) * vbar[k * plane + at[lab]];
          D[13 + t][k] = (mx[lab] ? mirror_sign(k, 0, 1) : 1.0) *
                         (my[lab] ? mirror_sign(k, 1, 1) : 1.0) * wbar[k * plane + at[lab]];
        }
      }
      int charwise = P->eq == EQ_EULER && P->char_decomp;
      int single = !charwise || P->char_decomp == 2; /* one reconstruction for both directions */
      int iface = charwise && P->char_decomp == 3;   /* edge values in interface bases */
      for (int sweep = 0; sweep < (single ? 1 : 2); ++sweep) {
        double pts[NPTS2][4], vh[4], wh[4];
        if (charwise) {
          if (project_recon_2d(P, D, D[4], sweep, nc, pts, vh, wh)) {
            bad |= 1;
            break;
          }
        } else {
          recon_components_2d(P, D, nc, pts, vh, wh);
        }
        if (iface) {
          /* edge values of the low and high side of this sweep's direction
           * in the bases of the Roe averages with the neighbours there
           * (cells 4 and 6 in x, 2 and 8 in y) */
          int lo = sweep == 0 ? 3 : 1, hi = sweep == 0 ? 5 : 7;
          if (ORACLE_PLANT == 5) {
            const int t = lo;
            lo = hi;
            hi = t;
          }
          const int e_lo = sweep == 0 ? 0 : 6, e_hi = sweep == 0 ? 3 : 9;
          double Ur[4], q[NPTS2][4], qv[4], qw[4];
          if ((ORACLE_PLANT == 5 ? roe_state(P, D[4], D[lo], 2, Ur)
                                 : roe_state(P, D[lo], D[4], 2, Ur)) ||
              project_recon_2d(P, D, Ur, sweep, nc, q, qv, qw)) {
            bad |= 1;
            break;
          }
          for (int e = 0; e < 3; ++e)
            for (int k = 0; k < nc; ++k) pts[e_lo + e][k] = q[e_lo + e][k];
          if ((ORACLE_PLANT == 5 ? roe_state(P, D[hi], D[4], 2, Ur)
                                 : roe_state(P, D[4], D[hi], 2, Ur)) ||
              project_recon_2d(P, D, Ur, sweep, nc, q, qv, qw)) {
            bad |= 1;
            break;
          }
          for (int e = 0; e < 3; ++e)
            for (int k = 0; k < nc; ++k) pts[e_hi + e][k] = q[e_hi + e][k];
        }
        int do_x = single || sweep == 0;
        int do_y = single || sweep == 1;
        if (do_x) {
          for (int e = 0; e < 6; ++e)
            for (int k = 0; k < nc; ++k) out->xe[e][k] = pts[e][k];
          for (int k = 0; k < nc; ++k) out->volf[k] = 0.0;
          for (int G = 0; G < 3; ++G)
            for (int H = 0; H < 3; ++H) {
              double f[4];
              phys_flux(P, 2, 0, pts[12 + 3 * G + H], f);
              for (int k = 0; k < nc; ++k) out->volf[k] += G3_W[G] * G3_W[H] * f[k];
            }
          for (int k = 0; k < nc; ++k) out->vh[k] = vh[k];
        }
        if (do_y) {
          for (int e = 0; e < 6; ++e)
            for (int k = 0; k < nc; ++k) out->ye[e][k] = pts[6 + e][k];
          for (int k = 0; k < nc; ++k) out->volg[k] = 0.0;
          for (int G = 0; G < 3; ++G)
            for (int H = 0; H < 3; ++H) {
              double g[4];
              phys_flux(P, 2, 1, pts[12 + 3 * G + H], g);
              for (int k = 0; k < nc; ++k) out->volg[k] += G3_W[G] * G3_W[H] * g[k];
            }
          for (int k = 0; k < nc; ++k) out->wh[k] = wh[k];
        }
      }
    }
  }
  if (bad) {
    free(C);
    return ERR_NONPHYSICAL;
  }
  /* fluxes and right-hand sides */
#pragma omp parallel for schedule(static) if (nx * ny >= ORACLE_OMP_MIN_2D)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const cell2d *c = C + (size_t)(j + 1) * ex + (i + 1);
      const cell2d *cl = c - 1, *cr = c + 1, *cb = c - ex, *ct = c + ex;
      double fl[3][4], fr[3][4], gb[3][4], gt[3][4];
      for (int G = 0; G < 3; ++G) {
        double a[4], b[4];
        /* x_{i-1/2}: u^- = left cell at +1/2, u^+ = this cell at -1/2 */
        phys_flux(P, 2, 0, cl->xe[3 + G], a);
        phys_flux(P, 2, 0, c->xe[G], b);
        for (int k = 0; k < nc; ++k)
          fl[G][k] = 0.5 * (a[k] + b[k] - alpha[0] * (c->xe[G][k] - cl->xe[3 + G][k]));
        phys_flux(P, 2, 0, c->xe[3 + G], a);
        phys_flux(P, 2, 0, cr->xe[G], b);
        for (int k = 0; k < nc; ++k)
          fr[G][k] = 0.5 * (a[k] + b[k] - alpha[0] * (cr->xe[G][k] - c->xe[3 + G][k]));
        /* y_{j-1/2}: u^- = bottom cell at eta=+1/2, u^+ = this cell at -1/2 */
        phys_flux(P, 2, 1, cb->ye[3 + G], a);
        phys_flux(P, 2, 1, c->ye[G], b);
        for (int k = 0; k < nc; ++k)
          gb[G][k] = 0.5 * (a[k] + b[k] - alpha[1] * (c->ye[G][k] - cb->ye[3 + G][k]));
        phys_flux(P, 2, 1, c->ye[3 + G], a);
        phys_flux(P, 2, 1, ct->ye[G], b);
        for (int k = 0; k < nc; ++k)
          gt[G][k] = 0.5 * (a[k] + b[k] - alpha[1] * (ct->ye[G][k] - c->ye[3 + G][k]));
      }
      for (int k = 0; k < nc; ++k) {
        double sx = 0, sy = 0, ax = 0, ay = 0, mx = 0, my = 0;
        for (int G = 0; G < 3; ++G) {
          sx += G3_W[G] * (fr[G][k] - fl[G][k]);
          sy += G3_W[G] * (gt[G][k] - gb[G][k]);
          ax += G3_W[G] * (fl[G][k] + fr[G][k]);
          ay += G3_W[G] * (gb[G][k] + gt[G][k]);
          mx += G3_W[G] * g3_nodes[G] * (fr[G][k] - fl[G][k]); /* eta_G weighted */
          my += G3_W[G] * g3_nodes[G] * (gt[G][k] - gb[G][k]); /* xi_G weighted  */
        }
        size_t o = k * plane + (size_t)j * nx + i;
        F1[o] = -sx / dx - sy / dy;
        F2[o] = -ax / (2.0 * dx) + c->volf[k] / dx - my / dy;
        F3[o] = -mx / dx - ay / (2.0 * dy) + c->volg[k] / dy;
        vhat[o] = c->vh[k];
        what[o] = c->wh[k];
      }
    }
  }
  free(C);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* wave speeds and validity                                                 */
/* ------------------------------------------------------------------------ */
/* alpha[d] = max over cells of |f'_d(u)| (Euler: |u_d| + c), d < dim. */
int oracle_max_wavespeed(const oracle_params *P, int dim, size_t ncell, const double *ubar,
                         double *alpha) {
  double a0 = 0.0, a1 = 0.0;
  for (size_t c = 0; c < ncell; ++c) {
    if (P->eq == EQ_ADVECTION) {
      a0 = fabs(P->adv_x);
      a1 = fabs(P->adv_y);
      break;
    }
    if (P->eq == EQ_BURGERS) {
      double s = fabs(ubar[c]);
      if (s > a0) a0 = s;
      if (s > a1) a1 = s;
      continue;
    }
    double U[4];
    for (int k = 0; k < P->ncomp; ++k) U[k] = ubar[(size_t)k * ncell + c];
    if (!is_physical(P, dim, U)) return ERR_NONPHYSICAL;
    double rho = U[0];
    double q2 = 0.0;
    for (int d = 0; d < dim; ++d) q2 += U[1 + d] * U[1 + d];
    double p = (P->gas_gamma - 1.0) * (U[dim + 1] - 0.5 * q2 / rho);
    double cs = sqrt(P->gas_gamma * p / rho);
    double s0 = fabs(U[1] / rho) + cs;
    if (s0 > a0) a0 = s0;
    if (dim == 2) {
      double s1 = fabs(U[2] / rho) + cs;
      if (s1 > a1) a1 = s1;
    }
  }
  alpha[0] = a0;
  alpha[1] = a1;
  return 0;
}

/* 1 if every cell average is a valid state */
int oracle_all_physical(const oracle_params *P, int dim, size_t ncell, const double *ubar) {
  for (size_t c = 0; c < ncell; ++c) {
    double U[4];
    for (int k = 0; k < P->ncomp; ++k) U[k] = ubar[(size_t)k * ncell + c];
    if (!is_physical(P, dim, U)) return 0;
  }
  return 1;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of later calls (timing only; results do not depend on it). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
