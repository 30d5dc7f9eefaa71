// One fused HWENO-U Runge-Kutta stage in 2D (Section 2.2): the true-2D
// quartic reconstruction on the 3x3 stencil (Step 1), smoothness indicators
// and scale-invariant weights (Steps 2-3), the modified moments v^, w^, the
// 21 point values, Lax-Friedrichs fluxes at the 3 Gauss points of every
// edge, the right-hand sides F1, F2, F3 of Eq. (2.16) and the modified
// SSP-RK3 update (Step 4).
//
// Euler: the reconstruction runs on local characteristic variables in two
// direction-split sweeps (Remark 2.2).  The y-sweep projects the stencil with
// the eigenvectors of g' at the cell average and yields the y-edge values,
// the interior values used for g, and w^; the x-sweep does the same with f'
// for the x-edges, f and v^.  Each characteristic field is reconstructed
// independently and the combined polynomials are mapped back to conserved
// variables before they are evaluated.  Scalar laws (and component-wise
// Euler) use one reconstruction for both directions.
//
// Mapping: a wave (one 64-thread block) marches a strip of 62 output columns
// upward, one row per step; lane l holds column strip*62 - 1 + l (lanes 0 and
// 63 only supply the neighbour columns' x-edge values).  The three stencil
// rows live in a ring of LDS rows shared by the wave; the row after next is
// prefetched into registers while the current row is computed.  x-interface
// values and fluxes move between lanes by shuffles.  The upper y-edge values
// of the previous row and that row's partially accumulated right-hand side
// stay in registers, so every flux is evaluated once and every row written
// once.  Waves take balanced runs of (strip, rows) from a per-wave work list:
// one persistent launch covers one large grid or many instances of uneven
// size.
#include <algorithm>

#include "hwenou_internal.hpp"

namespace hwenou {

constexpr int kCols = 66;  // LDS columns: strip*62 - 2 .. strip*62 + 63

__device__ __forceinline__ double g3w(int g) { return g == 1 ? G3W1 : G3W0; }
__device__ __forceinline__ double g3x(int g) { return g == 0 ? -G3S : (g == 1 ? 0.0 : G3S); }

// Primitive quantities at the cell average shared by both sweeps.
struct Prim {
  double u, v, c, ci, H, b1, b2, q2;
};

template <class TR>
__device__ __forceinline__ Prim make_prim(double gm1, const double (&U)[4]) {
  Prim p;
  const double rinv = rcp_w<TR>(U[0]);
  p.u = U[1] * rinv;
  p.v = U[2] * rinv;
  p.q2 = p.u * p.u + p.v * p.v;
  const double pr = gm1 * (U[3] - 0.5 * U[0] * p.q2);
  const double c2 = (gm1 + 1.0) * pr * rinv;
  p.ci = rsq_w<TR>(c2);
  p.c = c2 * p.ci;
  p.H = (U[3] + pr) * rinv;
  p.b1 = gm1 * (p.ci * p.ci);
  p.b2 = 0.5 * p.b1 * p.q2;
  return p;
}

// The same quantities at the Roe average of two cell averages (the
// per-interface bases): sqrt(rho)-weighted velocity and total enthalpy,
// c^2 = (gamma - 1)(H - q^2 / 2).  The arguments come in a fixed order (the
// lower or left cell first), so the two cells that share an interface form
// bitwise the same basis.
template <class TR>
__device__ __forceinline__ Prim make_prim_roe(double gm1, const double (&UL)[4],
                                              const double (&UR)[4]) {
  Prim p;
  const double il = rsq_w<TR>(UL[0]), ir = rsq_w<TR>(UR[0]);  // 1/sqrt(rho)
  const double sl = UL[0] * il, sr = UR[0] * ir;                 // sqrt(rho)
  const double w = rcp_w<TR>(sl + sr);
  p.u = (UL[1] * il + UR[1] * ir) * w;
  p.v = (UL[2] * il + UR[2] * ir) * w;
  p.q2 = p.u * p.u + p.v * p.v;
  // sqrt(rho) H = (E + p) / sqrt(rho), with p = (gamma - 1)(E - |m|^2 / (2 rho))
  const double hl = (UL[3] + gm1 * (UL[3] - 0.5 * (UL[1] * UL[1] + UL[2] * UL[2]) * il * il)) * il;
  const double hr = (UR[3] + gm1 * (UR[3] - 0.5 * (UR[1] * UR[1] + UR[2] * UR[2]) * ir * ir)) * ir;
  p.H = (hl + hr) * w;
  const double c2 = gm1 * (p.H - 0.5 * p.q2);
  p.ci = rsq_w<TR>(c2);
  p.c = c2 * p.ci;
  p.b1 = gm1 * (p.ci * p.ci);
  p.b2 = 0.5 * p.b1 * p.q2;
  return p;
}

// Row k of the left eigenvectors and column k of the right eigenvectors of
// the Euler flux Jacobian in direction DIR (ideal gas):
// x: R = [(1,u-c,v,H-uc), (1,u,v,q^2/2), (0,0,1,v), (1,u+c,v,H+uc)]
// y: R = [(1,u,v-c,H-vc), (1,u,v,q^2/2), (0,1,0,u), (1,u,v+c,H+vc)]
template <int DIR>
__device__ __forceinline__ void eig_row(const Prim& p, int k, double (&l)[4], double (&r)[4]) {
  const double un = DIR == 0 ? p.u : p.v;  // normal velocity
  const double ut = DIR == 0 ? p.v : p.u;  // tangential velocity
  const int n = DIR == 0 ? 1 : 2, t = DIR == 0 ? 2 : 1;
  double ll[4], rr[4];
  if (k == 0 || k == 3) {
    const double s = k == 0 ? 1.0 : -1.0;
    ll[0] = 0.5 * (p.b2 + s * un * p.ci);
    ll[n] = -0.5 * (p.b1 * un + s * p.ci);
    ll[t] = -0.5 * p.b1 * ut;
    ll[3] = 0.5 * p.b1;
    rr[0] = 1.0;
    rr[n] = un - s * p.c;
    rr[t] = ut;
    rr[3] = p.H - s * un * p.c;
  } else if (k == 1) {
    ll[0] = 1.0 - p.b2;
    ll[n] = p.b1 * un;
    ll[t] = p.b1 * ut;
    ll[3] = -p.b1;
    rr[0] = 1.0;
    rr[n] = un;
    rr[t] = ut;
    rr[3] = 0.5 * p.q2;
  } else {
    ll[0] = -ut;
    ll[n] = 0.0;
    ll[t] = 1.0;
    ll[3] = 0.0;
    rr[0] = 0.0;
    rr[n] = 0.0;
    rr[t] = 1.0;
    rr[3] = ut;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    l[m] = ll[m];
    r[m] = rr[m];
  }
}

template <int NC, class TM>
struct RowBuf {
  double u[3][NC][kCols];      // cell averages of three rows
  double m[3][2][NC][kCols];   // x and y moments of three rows (widened once on store)
};

// The 17 stencil values of field/component data around lane column `l`
// (LDS columns l, l+1, l+2; ring slots sb, sc, st for rows j-1, j, j+1).
template <int NC, class TM>
__device__ __forceinline__ void read_stencil(const RowBuf<NC, TM>& B, int sb, int sc, int st, int l,
                                             int k, Sten2& S) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S.u[a] = B.u[sb][k][l + a];
    S.u[3 + a] = B.u[sc][k][l + a];
    S.u[6 + a] = B.u[st][k][l + a];
  }
  S.v[0] = B.m[sb][0][k][l + 1];
  S.v[1] = B.m[sc][0][k][l];
  S.v[2] = B.m[sc][0][k][l + 2];
  S.v[3] = B.m[st][0][k][l + 1];
  S.w[0] = B.m[sb][1][k][l + 1];
  S.w[1] = B.m[sc][1][k][l];
  S.w[2] = B.m[sc][1][k][l + 2];
  S.w[3] = B.m[st][1][k][l + 1];
}

// Scalar HWENO reconstruction of one stencil -> combined coefficients
template <class TR, bool SI, bool FOLD = false>
__device__ __forceinline__ void recon_scalar(const SchemeParams& P, const Sten2& S, TR (&C)[15],
                                             double* a_out = nullptr) {
  double c[15];
  p0_coeffs_2d(S, c);
  const double u5 = S.u[4];
  const double asum = fabs(S.u[1]) + fabs(S.u[3]) + fabs(u5) + fabs(S.u[5]) + fabs(S.u[7]);
  hweno_2d<TR, SI, FOLD>(P, c, u5, u5 - S.u[3], S.u[5] - u5, u5 - S.u[1], S.u[7] - u5, asum, C,
                         a_out);
}

// One characteristic field K of the sweep in direction DIR: project the
// stencil with row K of L and reconstruct.  Returns C (C[0..2] combined
// coefficients, C[3..14] p0 coefficients) and the factor a of p0.  The shear
// field (K = 2) has only two non-zero entries in its L row; they are used
// directly.
template <int DIR, int K, bool SI, class TR, class TM>
__device__ __forceinline__ void char_field(const SchemeParams& P, const Prim& pr,
                                           const RowBuf<4, TM>& B, int sb, int sc, int st, int l,
                                           TR (&C)[15], double& a) {
  double lrow[4], rcol[4];
  eig_row<DIR>(pr, K, lrow, rcol);
  Sten2 W;
  if constexpr (K == 2) {
    // L row: -u_t at density, 1 at the tangential momentum
    constexpr int t = DIR == 0 ? 2 : 1;
    Sten2 S0, St;
    read_stencil<4, TM>(B, sb, sc, st, l, 0, S0);
    read_stencil<4, TM>(B, sb, sc, st, l, t, St);
    const double m0 = lrow[0];
#pragma unroll
    for (int q = 0; q < 9; ++q) W.u[q] = St.u[q] + m0 * S0.u[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      W.v[q] = St.v[q] + m0 * S0.v[q];
      W.w[q] = St.w[q] + m0 * S0.w[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) W.u[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) W.v[q] = W.w[q] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      Sten2 S;
      read_stencil<4, TM>(B, sb, sc, st, l, m, S);
      const double lm = lrow[m];
#pragma unroll
      for (int q = 0; q < 9; ++q) W.u[q] += lm * S.u[q];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        W.v[q] += lm * S.v[q];
        W.w[q] += lm * S.w[q];
      }
    }
  }
  recon_scalar<TR, SI, true>(P, W, C, &a);
}

// Characteristic sweep in direction DIR: combined polynomials of the four
// fields mapped back to conserved variables, Cc[m][n] = sum_K R[m][K] P_K[n].
// Each field's polynomial P_K arrives as C with C[0..2] combined and C[3..14]
// still to be scaled by the factor a of its p0.  The right eigenvectors
//   r0 = (1, un - c, ut, H - un c), r1 = (1, un, ut, q^2/2),
//   r2 = (0, 0, 1, ut),             r3 = (1, un + c, ut, H + un c)
// (components: density, normal momentum, tangential momentum, energy) give
//   Cc_rho = S + P1,          S = P0 + P3,  D = P3 - P0,
//   Cc_n   = un Cc_rho + c D,
//   Cc_t   = ut Cc_rho + P2,
//   Cc_E   = H S + un c D + q^2/2 P1 + ut P2,
// so the fields are taken in the order 0, 3, 1, 2 and fold into S, D and
// then into Cc.  The entropy field (K = 1) has the same left row and right
// column in both directions: its polynomial is reconstructed once per cell
// (by the first sweep) and passed to the second through LDS (PARK: a second
// sweep follows).  OVERLAP12: no scheduling barrier between fields 1 and 2
// (the FP64 split sweeps fit their registers without it and run 0.7% faster;
// the other kernels then spill or run slower).
template <int DIR, bool SI, bool PARK, class TR, class TM, bool OVERLAP12 = false>
__device__ __forceinline__ void char_sweep(const SchemeParams& P, const Prim& pr,
                                           const RowBuf<4, TM>& B, int sb, int sc, int st, int l,
                                           TR (&Cc)[4][15], TR (*c1buf)[64], bool have_c1) {
  constexpr int nd = DIR == 0 ? 1 : 2, td = DIR == 0 ? 2 : 1;  // normal, tangential momentum
  const double un = DIR == 0 ? pr.u : pr.v, ut = DIR == 0 ? pr.v : pr.u;
  TR C[15], S[15], D[15];
  double a;
  char_field<DIR, 0, SI, TR, TM>(P, pr, B, sb, sc, st, l, C, a);
  {
    const TR a0 = (TR)a;
#pragma unroll
    for (int n = 0; n < 15; ++n) S[n] = n < 3 ? C[n] : a0 * C[n];  // P0
  }
  char_field<DIR, 3, SI, TR, TM>(P, pr, B, sb, sc, st, l, C, a);
  {
    const TR a3 = (TR)a;
#pragma unroll
    for (int n = 0; n < 15; ++n) {
      const TR p0 = S[n];
      const TR f = n < 3 ? (TR)1 : a3;
      S[n] = f * C[n] + p0;
      D[n] = f * C[n] - p0;
    }
  }
  // scheduling barriers keep the later fields apart (bounds register pressure;
  // without them the compiler spills to scratch)
  __builtin_amdgcn_sched_barrier(0);
  {
    TR C1[15];
    double a1;
    if (!have_c1) {
      char_field<DIR, 1, SI, TR, TM>(P, pr, B, sb, sc, st, l, C1, a1);
      if constexpr (PARK) {  // parked in LDS for the other sweep
#pragma unroll
        for (int n = 0; n < 15; ++n) c1buf[n][l] = C1[n];
        c1buf[15][l] = (TR)a1;
      }
    } else {
#pragma unroll
      for (int n = 0; n < 15; ++n) C1[n] = c1buf[n][l];
      a1 = (double)c1buf[15][l];
    }
    const TR tun = (TR)un, tc = (TR)pr.c, tH = (TR)pr.H, tunc = (TR)(un * pr.c);
    const TR ta1 = (TR)a1, th = (TR)(0.5 * pr.q2), tha1 = (TR)(0.5 * pr.q2 * a1);
#pragma unroll
    for (int n = 0; n < 15; ++n) {
      const TR f1 = n < 3 ? (TR)1 : ta1, fh = n < 3 ? th : tha1;
      Cc[0][n] = f1 * C1[n] + S[n];
      Cc[nd][n] = tun * Cc[0][n] + tc * D[n];
      Cc[3][n] = fh * C1[n] + (tunc * D[n] + tH * S[n]);
    }
  }
  if constexpr (!OVERLAP12) __builtin_amdgcn_sched_barrier(0);
  char_field<DIR, 2, SI, TR, TM>(P, pr, B, sb, sc, st, l, C, a);
  {
    const TR tut = (TR)ut, a2 = (TR)a, uta2 = (TR)(ut * a);
#pragma unroll
    for (int n = 0; n < 15; ++n) {
      const TR f2 = n < 3 ? (TR)1 : a2, fu = n < 3 ? tut : uta2;
      Cc[td][n] = f2 * C[n] + tut * Cc[0][n];
      Cc[3][n] += fu * C[n];
    }
  }
}

// CHAR (Euler): 0 component-wise; 1 direction-split characteristic sweeps;
// 2 one reconstruction in x-characteristic variables for every output;
// 3 as 1, with the edge values at each interface reconstructed in the basis
// of the Roe average of the two cells that share it (three reconstructions
// per cell and direction: low interface, high interface, own average for the
// interior values and the moment).
// SI: scale-invariant weights compiled in (else the mode comes from P).
// ST: the Runge-Kutta stage (0, 1, 2), so that its coefficients and the
// stage-0-only stores are compiled in.
// One wave per block and one resident wave per SIMD (the row state needs
// 256 VGPRs plus 85-252 AGPRs).
template <int EQ, int CHAR, bool SI, int ST, class TR, class TM>
__global__ __launch_bounds__(64, 1) void stage2d_kernel(const StageArgs<TM> A) {
  constexpr int NC = EQ == EQ_EULER ? 4 : 1;
  constexpr bool PROJ = EQ == EQ_EULER && CHAR != 0;   // characteristic variables
  constexpr bool SPLIT = EQ == EQ_EULER && (CHAR == 1 || CHAR == 3);  // an x-direction sweep
  constexpr bool IFACE = EQ == EQ_EULER && CHAR == 3;  // interface bases for edge values
  __shared__ RowBuf<NC, TM> B;
  __shared__ TR c1buf[16][64];  // entropy-field polynomial shared by the two sweeps
  // per-interface bases: the edge values of the low and the high edge of the
  // current direction, parked while the cell's own basis is reconstructed
  __shared__ TR ebuf[IFACE ? 2 * 3 * NC : 1][64];
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  if (w >= A.n_waves) return;
  const SchemeParams& P = A.P;
  // out = ra * base + rb * (in + dt F)
  constexpr double ra = ST == 0 ? 0.0 : (ST == 1 ? 0.75 : 1.0 / 3.0);
  constexpr double rb = ST == 0 ? 1.0 : (ST == 1 ? 0.25 : 2.0 / 3.0);
  const long long plane = A.plane;
  const double gm1 = P.gas_gamma - 1.0;

  for (int it = A.work_ptr[w]; it < A.work_ptr[w + 1]; ++it) {
    const WorkItem wk = A.work[it];
    if (A.done != nullptr && A.done[wk.inst]) continue;
    const InstDev I = A.inst[wk.inst];
    const int nx = I.nx, ny = I.ny;
    const int c0 = wk.a * kStripWidth;
    int i = c0 - 1 + lane;
    if (i > nx) i = nx;
    const bool col_owner = lane >= 1 && lane <= kStripWidth && i < nx;
    // byte offsets of this lane's column in a row (clamped into the row, so
    // that loads need no lane mask; only owners store)
    const int ic = min(max(i, 0), nx - 1);
    const unsigned ou = (unsigned)ic * 8u, om = (unsigned)ic * (unsigned)sizeof(TM);
    const TR a1 = (TR)A.alpha[2 * wk.inst], a2 = (TR)A.alpha[2 * wk.inst + 1];
    const double dt = A.dt[wk.inst];
    const double idx = 1.0 / I.dx, idy = 1.0 / I.dy;
    const int r0 = wk.b, r1 = wk.c;
    const double* u_in = A.u_in + I.offset;
    const TM* m_in = A.m_in + I.offset;

    // grid columns of the LDS columns this lane loads (clamped, then wrapped)
    const int gx0 = wrap_index(min(c0 - 2 + lane, nx + 1), nx, I.bc[0], I.bc[1]);
    const int gx1 = wrap_index(min(c0 + 62 + lane, nx + 1), nx, I.bc[0], I.bc[1]);
    const bool walls = EQ == EQ_EULER && (I.bc[0] == BC_REFLECTIVE || I.bc[1] == BC_REFLECTIVE ||
                                          I.bc[2] == BC_REFLECTIVE || I.bc[3] == BC_REFLECTIVE);
    const bool extra = lane < 2;
    const unsigned o0u = (unsigned)gx0 * 8u, o0m = (unsigned)gx0 * (unsigned)sizeof(TM);
    const unsigned o1u = (unsigned)gx1 * 8u, o1m = (unsigned)gx1 * (unsigned)sizeof(TM);

    // register prefetch of one row (this lane's column and, for lanes 0-1,
    // one of the two extra columns)
    double pu0[NC], pu1[NC];
    TM pm0[2][NC], pm1[2][NC];
    auto fetch = [&](int row) {
      const long long base = (long long)wrap_index(row, ny, I.bc[2], I.bc[3]) * nx;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const double* pu = u_in + (k * plane + base);
        const TM* pv = m_in + (k * plane + base);
        const TM* pw = m_in + ((NC + k) * plane + base);
        pu0[k] = load_at(pu, o0u);
        pm0[0][k] = load_at(pv, o0m);
        pm0[1][k] = load_at(pw, o0m);
        if (extra) {
          pu1[k] = load_at(pu, o1u);
          pm1[0][k] = load_at(pv, o1m);
          pm1[1][k] = load_at(pw, o1m);
        }
      }
    };
    // Reflective walls: the stored cells of grid row `row` that are mirror
    // images (ghost columns beyond an x-wall, or the whole row beyond a
    // y-wall) get the signs of the mirror image: the wall-normal momentum
    // and the moments along the wall normal change sign (twice for the x-
    // moment of the x-momentum and the y-moment of the y-momentum).  Runs
    // after the row is in LDS, outside the register-heavy part of the row.
    auto mirror_row = [&](int slot, int row) {
      const bool my = (row < 0 && I.bc[2] == BC_REFLECTIVE) ||
                      (row >= ny && I.bc[3] == BC_REFLECTIVE);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (e == 1 && !extra) break;
        const int c = e == 0 ? c0 - 2 + lane : c0 + 62 + lane;  // grid column
        const bool mx = (c < 0 && I.bc[0] == BC_REFLECTIVE) ||
                        (c >= nx && I.bc[1] == BC_REFLECTIVE);
        if (!(mx || my)) continue;
        const int l = e == 0 ? lane : 64 + lane;
        double uu[NC], mm[2][NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          uu[k] = B.u[slot][k][l];
          mm[0][k] = B.m[slot][0][k][l];
          mm[1][k] = B.m[slot][1][k][l];
        }
        if (mx) mirror_cell<0, NC>(uu, mm, 2);
        if (my) mirror_cell<1, NC>(uu, mm, 2);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          B.u[slot][k][l] = uu[k];
          B.m[slot][0][k][l] = mm[0][k];
          B.m[slot][1][k][l] = mm[1][k];
        }
      }
    };
    auto store = [&](int slot, int row) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        B.u[slot][k][lane] = pu0[k];
        B.m[slot][0][k][lane] = (double)pm0[0][k];
        B.m[slot][1][k][lane] = (double)pm0[1][k];
        if (extra) {
          B.u[slot][k][64 + lane] = pu1[k];
          B.m[slot][0][k][64 + lane] = (double)pm1[0][k];
          B.m[slot][1][k][64 + lane] = (double)pm1[1][k];
        }
      }
      if constexpr (EQ == EQ_EULER) {
        if (walls) mirror_row(slot, row);
      }
    };
    __syncthreads();  // the previous item's reads of B are complete
    // prologue: rows r0-2 .. r0 into ring slots 0..2, r0+1 into registers
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      fetch(r0 - 2 + q);
      store(q, r0 - 2 + q);
    }
    fetch(r0 + 1);
    __syncthreads();

    // state carried from the row below (pending right-hand side of row j-1)
    TR yprev[3][NC];
    double F1p[NC];
    TR F2p[NC], F3p[NC], vhp[NC], whp[NC];
    double amax_x = 0.0, amax_y = 0.0;
    bool ok = true;

    int sb = 0, sc = 1, st = 2;  // ring slots of rows j-1, j, j+1
    for (int j = r0 - 1; j <= r1; ++j) {
      const bool row_out = j >= r0 && j < r1;
      const bool fin = j - 1 >= r0 && j - 1 < r1;  // row j-1 is finished in this step

      // base (u^n, v^n, w^n) of row j-1, loaded now and used after the y-sweep
      double ubase[NC];
      TM vbase[NC], wbase[NC];
      const long long orow = I.offset + (long long)(j - 1) * nx;  // row j-1
      if (ST != 0 && fin) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          ubase[k] = load_at(A.u_base + (k * plane + orow), ou);
          vbase[k] = load_at(A.m_base + (k * plane + orow), om);
          wbase[k] = load_at(A.m_base + ((NC + k) * plane + orow), om);
        }
      }

      // ---- reconstruction of row j, y-direction ----
      TR Cc[NC][15];
      Prim pr;
      if constexpr (IFACE) {
        auto roe_rows = [&](int sl, int sr) {  // Roe basis of rows sl (below) and sr (above)
          double UL[4], UR[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            UL[k] = B.u[sl][k][lane + 1];
            UR[k] = B.u[sr][k][lane + 1];
          }
          return make_prim_roe<TR>(gm1, UL, UR);
        };
        // top edge, eta = +1/2, in the basis of y_{j+1/2}
        char_sweep<1, SI, false, TR, TM>(P, roe_rows(sc, st), B, sb, sc, st, lane, Cc, c1buf,
                                         false);
#pragma unroll
        for (int G = 0; G < 3; ++G)
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            TR d[5], e0, e1, g0, g1, g2;
            restrict_xi_line<TR>(Cc[k], G, d);
            eval5<TR>(d, e0, e1, g0, g1, g2);
            ebuf[(3 + G) * NC + k][lane] = e1;
          }
        __builtin_amdgcn_sched_barrier(0);
        if (j >= r0) {
          // bottom edge, eta = -1/2, in the basis of y_{j-1/2}
          char_sweep<1, SI, false, TR, TM>(P, roe_rows(sb, sc), B, sb, sc, st, lane, Cc, c1buf,
                                           false);
#pragma unroll
          for (int G = 0; G < 3; ++G)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
              TR d[5], e0, e1, g0, g1, g2;
              restrict_xi_line<TR>(Cc[k], G, d);
              eval5<TR>(d, e0, e1, g0, g1, g2);
              ebuf[G * NC + k][lane] = e0;
            }
          __builtin_amdgcn_sched_barrier(0);
          // interior values and w^ in the cell's own basis
          double U5[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) U5[k] = B.u[sc][k][lane + 1];
          pr = make_prim<TR>(gm1, U5);
          char_sweep<1, SI, true, TR, TM>(P, pr, B, sb, sc, st, lane, Cc, c1buf, false);
        }
      } else if constexpr (PROJ) {
        double U5[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) U5[k] = B.u[sc][k][lane + 1];
        pr = make_prim<TR>(gm1, U5);
        char_sweep<SPLIT ? 1 : 0, SI, SPLIT, TR, TM, SPLIT && sizeof(TR) == 8>(
            P, pr, B, sb, sc, st, lane, Cc, c1buf, false);
      } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          Sten2 S;
          read_stencil<NC, TM>(B, sb, sc, st, lane, k, S);
          recon_scalar<TR, SI>(P, S, Cc[k]);
        }
      }
      // y-edges at (xi_G, -+1/2), interior values for g (and f when the
      // reconstruction is shared), y-fluxes at y_{j-1/2}
      TR F1n_s[NC], F2n[NC], F3n[NC];  // new row: bottom-flux terms
      double F1n[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        F1n[k] = 0.0;
        F2n[k] = (TR)0;
        F3n[k] = (TR)0;
        F1n_s[k] = (TR)0;
      }
      TR volf[NC], volg[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) volf[k] = volg[k] = (TR)0;
#pragma unroll
      for (int G = 0; G < 3; ++G) {
        const TR xg = (TR)g3x(G);
        TR ym[NC], yp[NC], in[3][NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          TR d[5];
          restrict_xi_line<TR>(Cc[k], G, d);
          eval5<TR>(d, ym[k], yp[k], in[0][k], in[1][k], in[2][k]);
          if constexpr (IFACE) {
            ym[k] = ebuf[G * NC + k][lane];
            yp[k] = ebuf[(3 + G) * NC + k][lane];
          }
        }
        if (row_out) {
#pragma unroll
          for (int H = 0; H < 3; ++H) {
            const TR wgt = (TR)(g3w(G) * g3w(H));
            TR g[NC];
            phys_flux<EQ, NC, 1, TR>(P, in[H], g);
#pragma unroll
            for (int k = 0; k < NC; ++k) volg[k] += wgt * g[k];
            if constexpr (!SPLIT) {
              TR f[NC];
              phys_flux<EQ, NC, 0, TR>(P, in[H], f);
#pragma unroll
              for (int k = 0; k < NC; ++k) volf[k] += wgt * f[k];
            }
          }
        }
        if (j >= r0) {
          // u- = row below at eta = +1/2, u+ = this row at eta = -1/2
          TR gb[NC];
          lf_flux2<EQ, NC, 1, TR>(P, yprev[G], ym, a2, gb);  // twice the flux
          const TR wg = (TR)(0.5 * g3w(G));
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            F1n_s[k] += wg * gb[k];       // sum_G w_G g_{G,j-1/2}
            if (G != 1) F2n[k] += wg * xg * gb[k];  // sum_G w_G xi_G g_{G,j-1/2} (xi_1 = 0)
          }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) yprev[G][k] = yp[k];
      }
      if (j >= r0) {
        // the same sums close row j-1 (upper edge) and open row j (lower edge)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          F1p[k] -= (double)F1n_s[k] * idy;
          F2p[k] -= F2n[k] * (TR)idy;
          F3p[k] -= F1n_s[k] * (TR)(0.5 * idy);
          F3n[k] = -F1n_s[k] * (TR)(0.5 * idy);
          F2n[k] = F2n[k] * (TR)idy;
        }
      }
      TR whn[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) whn[k] = qw_2d<TR>(Cc[k]);

      // ---- row j-1 is complete: Runge-Kutta update and store ----
      if (fin) {
        if (col_owner) {
          double Uo[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            const double uin = B.u[sb][k][lane + 1];
            const double ub = ST == 0 ? 0.0 : ubase[k];
            const double un = ra * ub + rb * (uin + dt * F1p[k]);
            TR vn, wn;
            if (ST == 0) {
              store_at(A.m_base + (k * plane + orow), om, (TM)vhp[k]);
              store_at(A.m_base + ((NC + k) * plane + orow), om, (TM)whp[k]);
              vn = vhp[k] + (TR)dt * F2p[k];
              wn = whp[k] + (TR)dt * F3p[k];
            } else {
              const TR vb = (TR)vbase[k];
              const TR wb = (TR)wbase[k];
              vn = (TR)ra * vb + (TR)rb * (vhp[k] + (TR)dt * F2p[k]);
              wn = (TR)ra * wb + (TR)rb * (whp[k] + (TR)dt * F3p[k]);
            }
            store_at(A.u_out + (k * plane + orow), ou, un);
            store_at(A.m_out + (k * plane + orow), om, (TM)vn);
            store_at(A.m_out + ((NC + k) * plane + orow), om, (TM)wn);
            Uo[k] = un;
          }
          if constexpr (ST == 2) {  // the wave speeds feed the next step's alpha
            double sx, sy;
            ok = wave_speeds<EQ, NC>(P, Uo, sx, sy) && ok;
            amax_x = fmax(amax_x, sx);
            amax_y = fmax(amax_y, sy);
          } else {
            ok = physical_state<EQ, NC>(Uo) && ok;
          }
        }
      }

      if (row_out) {
        // ---- x-direction reconstruction of row j ----
        if constexpr (IFACE) {
          auto roe_cols = [&](int cl) {  // Roe basis of columns cl (left) and cl + 1
            double UL[4], UR[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              UL[k] = B.u[sc][k][lane + cl];
              UR[k] = B.u[sc][k][lane + cl + 1];
            }
            return make_prim_roe<TR>(gm1, UL, UR);
          };
          // left edge, xi = -1/2, in the basis of x_{i-1/2}
          char_sweep<0, SI, false, TR, TM>(P, roe_cols(0), B, sb, sc, st, lane, Cc, c1buf,
                                           false);
#pragma unroll
          for (int H = 0; H < 3; ++H)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
              TR d[5], e0, e1, g0, g1, g2;
              restrict_eta_line<TR>(Cc[k], H, d);
              eval5<TR>(d, e0, e1, g0, g1, g2);
              ebuf[H * NC + k][lane] = e0;
            }
          __builtin_amdgcn_sched_barrier(0);
          // right edge, xi = +1/2, in the basis of x_{i+1/2}
          char_sweep<0, SI, false, TR, TM>(P, roe_cols(1), B, sb, sc, st, lane, Cc, c1buf,
                                           false);
#pragma unroll
          for (int H = 0; H < 3; ++H)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
              TR d[5], e0, e1, g0, g1, g2;
              restrict_eta_line<TR>(Cc[k], H, d);
              eval5<TR>(d, e0, e1, g0, g1, g2);
              ebuf[(3 + H) * NC + k][lane] = e1;
            }
          __builtin_amdgcn_sched_barrier(0);
          double U5[4];  // the own primitives again (cheaper than keeping them live)
#pragma unroll
          for (int k = 0; k < 4; ++k) U5[k] = B.u[sc][k][lane + 1];
          pr = make_prim<TR>(gm1, U5);
        }
        if constexpr (SPLIT)
          char_sweep<0, SI, false, TR, TM, !IFACE && sizeof(TR) == 8>(P, pr, B, sb, sc, st, lane,
                                                                      Cc, c1buf, true);
        double F1x[NC];
        TR F2x[NC], F3x[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          F1x[k] = 0.0;
          F2x[k] = F3x[k] = (TR)0;
        }
#pragma unroll
        for (int H = 0; H < 3; ++H) {
          const TR yh = (TR)g3x(H);
          TR xm[NC], xp[NC], in[3][NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            TR d[5];
            restrict_eta_line<TR>(Cc[k], H, d);
            eval5<TR>(d, xm[k], xp[k], in[0][k], in[1][k], in[2][k]);
            if constexpr (IFACE) {
              xm[k] = ebuf[H * NC + k][lane];
              xp[k] = ebuf[(3 + H) * NC + k][lane];
            }
          }
          if constexpr (SPLIT) {
#pragma unroll
            for (int G = 0; G < 3; ++G) {
              TR f[NC];
              phys_flux<EQ, NC, 0, TR>(P, in[G], f);
              const TR wgt = (TR)(g3w(G) * g3w(H));
#pragma unroll
              for (int k = 0; k < NC; ++k) volf[k] += wgt * f[k];
            }
          }
          // x_{i-1/2} at eta_H: u- = left lane at +1/2, u+ = this lane at -1/2
          TR um[NC], fl[NC], fr[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) um[k] = from_prev(xp[k]);
          lf_flux2<EQ, NC, 0, TR>(P, um, xm, a1, fl);  // twice the flux
#pragma unroll
          for (int k = 0; k < NC; ++k) fr[k] = from_next(fl[k]);
          const TR wg = (TR)(0.5 * g3w(H));
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            F1x[k] += (double)wg * ((double)fr[k] - (double)fl[k]);
            F2x[k] += wg * (fl[k] + fr[k]);
            if (H != 1) F3x[k] += wg * yh * (fr[k] - fl[k]);  // eta_1 = 0
          }
        }
        // pending right-hand side of row j
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          F1p[k] = -F1x[k] * idx + (double)F1n_s[k] * idy;
          F2p[k] = -F2x[k] * (TR)(0.5 * idx) + volf[k] * (TR)idx + F2n[k];
          F3p[k] = -F3x[k] * (TR)idx + volg[k] * (TR)idy + F3n[k];
          vhp[k] = qv_2d<TR>(Cc[k]);
          whp[k] = whn[k];
        }
      }

      // ---- advance the LDS ring: row j+2 from registers, prefetch j+3 ----
      __syncthreads();
      if (j + 2 <= r1 + 1) store(sb, j + 2);  // row j-1's slot takes row j+2
      if (j + 3 <= r1 + 1) fetch(j + 3);
      __syncthreads();
      const int s0 = sb;
      sb = sc;
      sc = st;
      st = s0;
    }
    if (!ok) atomicOr(&A.status[wk.inst], 1);
    if (ST == 2 && A.alpha_next != nullptr) {
      const double mx = wave_max(amax_x), my = wave_max(amax_y);
      if (lane == 0) {
        double* acc = A.alpha_next + alpha_slot(wk.inst, blockIdx.x, A.alpha_slots);
        atomic_max_nonneg(acc, mx);
        atomic_max_nonneg(acc + 1, my);
      }
    }
  }
}

template <int EQ, int CHAR, bool SI, class TR, class TM>
static hipError_t launch(const void* args, int blocks, int threads, hipStream_t s) {
  const auto& a = *static_cast<const StageArgs<TM>*>(args);
  switch (a.stage) {
    case 0:
      hipLaunchKernelGGL((stage2d_kernel<EQ, CHAR, SI, 0, TR, TM>), dim3(blocks), dim3(threads), 0,
                         s, a);
      break;
    case 1:
      hipLaunchKernelGGL((stage2d_kernel<EQ, CHAR, SI, 1, TR, TM>), dim3(blocks), dim3(threads), 0,
                         s, a);
      break;
    default:
      hipLaunchKernelGGL((stage2d_kernel<EQ, CHAR, SI, 2, TR, TM>), dim3(blocks), dim3(threads), 0,
                         s, a);
  }
  return hipGetLastError();
}

template <bool SI, class TR>
static hipError_t launch_t(int eq, int char_mode, const void* args, int blocks, int threads,
                           hipStream_t s) {
  switch (eq) {
    case EQ_ADVECTION: return launch<EQ_ADVECTION, 0, SI, TR, TR>(args, blocks, threads, s);
    case EQ_BURGERS: return launch<EQ_BURGERS, 0, SI, TR, TR>(args, blocks, threads, s);
    default:
      if (char_mode == 3) return launch<EQ_EULER, 3, SI, TR, TR>(args, blocks, threads, s);
      if (char_mode == 2) return launch<EQ_EULER, 2, SI, TR, TR>(args, blocks, threads, s);
      return char_mode ? launch<EQ_EULER, 1, SI, TR, TR>(args, blocks, threads, s)
                       : launch<EQ_EULER, 0, SI, TR, TR>(args, blocks, threads, s);
  }
}

hipError_t launch_stage_2d(int eq, int char_mode, bool mixed, bool scale_invariant,
                           const void* args, int blocks, int threads, hipStream_t s) {
  if (scale_invariant)
    return mixed ? launch_t<true, float>(eq, char_mode, args, blocks, threads, s)
                 : launch_t<true, double>(eq, char_mode, args, blocks, threads, s);
  return mixed ? launch_t<false, float>(eq, char_mode, args, blocks, threads, s)
               : launch_t<false, double>(eq, char_mode, args, blocks, threads, s);
}

template <int EQ, int CHAR, bool SI, int ST, class TR>
static int occupancy_st(int threads) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, stage2d_kernel<EQ, CHAR, SI, ST, TR, TR>, threads, 0) != hipSuccess)
    return 0;
  return blocks;
}

// resident blocks per CU common to the three stage kernels
template <int EQ, int CHAR, bool SI, class TR>
static int occupancy(int threads) {
  return std::min(occupancy_st<EQ, CHAR, SI, 0, TR>(threads),
                  std::min(occupancy_st<EQ, CHAR, SI, 1, TR>(threads),
                           occupancy_st<EQ, CHAR, SI, 2, TR>(threads)));
}

template <bool SI, class TR>
static int occupancy_t(int eq, int char_mode, int threads) {
  switch (eq) {
    case EQ_ADVECTION: return occupancy<EQ_ADVECTION, 0, SI, TR>(threads);
    case EQ_BURGERS: return occupancy<EQ_BURGERS, 0, SI, TR>(threads);
    default:
      if (char_mode == 3) return occupancy<EQ_EULER, 3, SI, TR>(threads);
      if (char_mode == 2) return occupancy<EQ_EULER, 2, SI, TR>(threads);
      return char_mode ? occupancy<EQ_EULER, 1, SI, TR>(threads)
                       : occupancy<EQ_EULER, 0, SI, TR>(threads);
  }
}

int occupancy_stage_2d(int eq, int char_mode, bool mixed, bool scale_invariant, int threads) {
  if (scale_invariant)
    return mixed ? occupancy_t<true, float>(eq, char_mode, threads)
                 : occupancy_t<true, double>(eq, char_mode, threads);
  return mixed ? occupancy_t<false, float>(eq, char_mode, threads)
               : occupancy_t<false, double>(eq, char_mode, threads);
}

}  // namespace hwenou
