// Device-side building blocks of the HWENO-U stage operator for gfx950.
//
// Everything here follows Section 2 of Fan, Qiu & Zhao, "A moment-based
// Hermite WENO scheme with unified stencils for hyperbolic conservation
// laws" (arXiv 2402.03074):
//   * reconstruction coefficients of p0 (quartic) and p_m (linear): the
//     Appendix tables, with the 2D c_{0,4} u_1 entry taken as -7/22 (the
//     value the moment conditions give; the printed +7/22 breaks the
//     antisymmetry of the xi*eta coefficient under x -> -x);
//   * smoothness indicators: Eq. (2.9) in 1D with the first square read as
//     (c_{0,1} + c_{0,3}/4)^2, and the printed sum of squares of Eq. (2.20) in 2D;
//   * scale-invariant nonlinear weights, Eq. (2.10)-(2.11) / (2.21)-(2.22);
//   * reconstruction u_i(x) and the HWENO moment modification, Eq. (2.12) / (2.23),
//     written as one combined polynomial C = (w0/g0) p0 + sum_m (w_m - w0 g_m/g0) p_m;
//   * Lax-Friedrichs fluxes (Eq. (2.4)) and Euler eigenvectors (Remark 2.2).
// The types are templated so that the FP64 path and the mixed path (FP64
// coefficients / smoothness indicators / weights, FP32 point values and
// fluxes) share one code path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hwenou {

enum : int { EQ_ADVECTION = 0, EQ_BURGERS = 1, EQ_EULER = 2 };
enum : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2 };

// Gauss points on [-1/2, 1/2]: 3-point Gauss (sqrt(15)/10, weights 5/18, 4/9)
// and 4-point Gauss-Lobatto (1/2, sqrt(5)/10, weights 1/12, 5/12).
constexpr double G3S = 0.38729833462074168852;
constexpr double G3W0 = 5.0 / 18.0;
constexpr double G3W1 = 4.0 / 9.0;
constexpr double GL4S = 0.22360679774997896964;
constexpr double GL4W0 = 1.0 / 12.0;
constexpr double GL4W1 = 5.0 / 12.0;

// Runtime scheme parameters shared by every kernel.
struct SchemeParams {
  double adv_x, adv_y;  // advection velocity
  double gas_gamma;     // ratio of specific heats
  double gamma_low;     // linear weight of each linear polynomial
  double eps;           // epsilon of the nonlinear weights
  // weight mode as arithmetic factors (no selects in the kernels):
  // u_ave <- ave_mul u_ave + ave_add: (1, 0) scale-invariant, (0, 1) ZQ;
  // nonlin = 1 for nonlinear weights, 0 for linear weights (w = gamma)
  double ave_mul, ave_add;
  double nonlin;
};

// Source cell of index i of a grid of n >= 3 cells, -3 <= i <= n + 2:
// periodic wrap, transmissive copy of the boundary cell, or the mirror image
// at a reflective wall (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2, n+2 -> n-3),
// flagged in `mirrored`.
__device__ __forceinline__ int bc_index(int i, int n, int bc_lo, int bc_hi, bool& mirrored) {
  mirrored = false;
  if (i < 0) {
    if (bc_lo == BC_PERIODIC) return i + n;
    mirrored = bc_lo == BC_REFLECTIVE;
    return mirrored ? -1 - i : 0;
  }
  if (i >= n) {
    if (bc_hi == BC_PERIODIC) return i - n;
    mirrored = bc_hi == BC_REFLECTIVE;
    return mirrored ? 2 * n - 1 - i : n - 1;
  }
  return i;
}
__device__ __forceinline__ int wrap_index(int i, int n, int bc_lo, int bc_hi) {
  bool m;
  return bc_index(i, n, bc_lo, bc_hi, m);
}

// Euler data of a cell mirrored across a wall normal to direction D
// (reflective boundary): the normal momentum (component 1 + D) changes sign,
// and the moments along D change sign once more because their local
// coordinate does.  u: averages [NC]; m: moments [dim][NC] (m[0] along x).
template <int D, int NC, class T, class TM>
__device__ __forceinline__ void mirror_cell(T (&u)[NC], TM (*m)[NC], int dim) {
  if constexpr (NC > 1 + D) {  // Euler only (scalar laws have no walls)
    u[1 + D] = -u[1 + D];
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k != 1 + D) m[D][k] = -m[D][k];
    if (dim == 2) m[1 - D][1 + D] = -m[1 - D][1 + D];
  }
}

// Global memory access through a wave-uniform base pointer (row and
// component folded in with scalar arithmetic) and a 32-bit per-lane byte
// offset, which halves the registers that hold per-lane offsets.  Offsets
// stay below 2^32 bytes because an instance holds at most 2^29 cells.
template <class T>
__device__ __forceinline__ T load_at(const T* base, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void store_at(T* base, unsigned byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// ---------------------------------------------------------------------------
// reciprocals: the hardware estimate refined by Newton-Raphson steps
// r <- r + r (1 - x r).  Measured on gfx950 over 4M arguments in
// [1e-20, 1e20] against correctly rounded division: the FP64 estimate is
// within 4.6e-8 (relative), one step within 2.2e-15 (10 ulp), two steps
// exact; the FP32 estimate is within 1 ulp, one step exact.
//   rcp_nr(double): two steps (FP64 kernels, and wherever FP64 is kept);
//   rcp_w<TR>(double): the FP64 quantities of the reconstruction (weights,
//     primitive variables for the eigenvectors): two steps for TR = double,
//     one for the mixed form (TR = float), whose results are FP32;
//   rcp_nr(float): one step (the mixed form's fluxes).  The 1-ulp estimate
//     alone is not enough there: over the ~3700 steps of the 80-cell 1D
//     Euler accuracy test its rounding doubles the mixed form's error floor.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <class TR>
__device__ __forceinline__ double rcp_w(double x) {
  if constexpr (sizeof(TR) == 8) {
    return rcp_nr(x);
  } else {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
  }
}
// 1/sqrt(x) for the sound speed of the eigenvectors: the hardware estimate
// refined by Newton-Raphson steps y <- y (3/2 - x y^2 / 2), as many as rcp_w
// takes (two for TR = double, one for the mixed form).
template <class TR>
__device__ __forceinline__ double rsq_w(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < (sizeof(TR) == 8 ? 2 : 1); ++k) {
    const double g = x * y, h = 0.5 * y;
    y = fma(y, fma(-g, h, 0.5), y);
  }
  return y;
}
__device__ __forceinline__ float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// ---------------------------------------------------------------------------
// nonlinear weights (Step 3), returned as the combination factors
//   a   = w0 / g0          (factor of p0)
//   b_m = w_m - a g_m      (factor of p_m)
// so that u_i = a p0 + sum_m b_m p_m.  Always evaluated in FP64.
// SI = true compiles the scale-invariant weights alone (the default mode);
// SI = false takes the weight mode from P at run time.  SCALE: scale the
// denominators by a power of two before their products are formed (below);
// on in the scale-invariant 2D kernels and in every 1D kernel.  The 2D
// kernels that take the mode at run time (ZQ and linear weights) leave it
// out to stay within their register budget: with u_ave = 1 their
// denominators grow only like the square of the state, and the products stay
// in range for states up to ~1e30.
// ---------------------------------------------------------------------------
template <int NM, bool SI, class TR, bool SCALE = SI>
__device__ __forceinline__ void combine_factors(const SchemeParams& P, const double (&beta)[NM + 1],
                                                double u_ave, double& a, double (&b)[NM]) {
  // At run time the weight mode enters through exact arithmetic factors
  // (multiplications by 0 or 1), so that the reconstruction of a field stays
  // one basic block without selects.
  const double gl = P.gamma_low;
  const double g0 = 1.0 - NM * gl;
  if constexpr (!SI) u_ave = fma(u_ave, P.ave_mul, P.ave_add);
  double t = 0.0;
#pragma unroll
  for (int m = 1; m <= NM; ++m) t += fabs(beta[0] - beta[m]);
  t *= (1.0 / NM);
  double tau = t * t;
  // unnormalised weights gamma_m e_m with e_m = 1 + tau / d_m and
  // d_m = beta_m u_ave + eps, all scaled by D = prod_k d_k so that one
  // reciprocal serves every weight: D e_m = D + tau P_m, with P_m the product
  // of the d_k other than d_m (prefix times suffix products).  The weights are
  // ratios of these, so the scale cancels exactly.  Before the products are
  // formed, u_ave, eps and tau are scaled by 2^-E, with 2^E the binade of
  // d_0, the quartic's denominator: the scaled d_0 lies in [1, 2) and the
  // other d_m keep their ratios to it, so the products follow the spread of
  // the d_m (wherever the data are not smooth d_0 is the largest; on smooth
  // data all are of one size), not the magnitude of the state.  A power of
  // two commutes with every rounding, so the scaled d_m and tau are exactly
  // 2^-E times the unscaled ones and the weights are bitwise those of the
  // unscaled form wherever that form stays in range.  What can still leave
  // the range is a spread beyond ~1e70 between the d_m; the products of the
  // smallest d_m then underflow, and those belong to the weights that are
  // negligible.
  double ua_s = u_ave, eps_s = P.eps;
  if constexpr (SCALE) {
    const int E = __builtin_amdgcn_frexp_exp(fma(beta[0], u_ave, P.eps)) - 1;
    ua_s = ldexp(u_ave, -E);
    eps_s = ldexp(P.eps, -E);
    tau = ldexp(tau, -E);
  }
  double d[NM + 1];
#pragma unroll
  for (int m = 0; m <= NM; ++m) d[m] = fma(beta[m], ua_s, eps_s);
  double pre[NM + 1], suf[NM + 1];  // pre[m] = d_0 .. d_{m-1}, suf[m] = d_m .. d_NM
  pre[1] = d[0];
#pragma unroll
  for (int m = 2; m <= NM; ++m) pre[m] = pre[m - 1] * d[m - 1];
  suf[NM] = d[NM];
#pragma unroll
  for (int m = NM - 1; m >= 1; --m) suf[m] = d[m] * suf[m + 1];
  const double D = d[0] * suf[1];
  double e[NM + 1];
  e[0] = fma(tau, suf[1], D);
#pragma unroll
  for (int m = 1; m < NM; ++m) e[m] = fma(tau, pre[m] * suf[m + 1], D);
  e[NM] = fma(tau, pre[NM], D);
  double el = e[1];
#pragma unroll
  for (int m = 2; m <= NM; ++m) el += e[m];
  const double inv = rcp_w<TR>(fma(g0, e[0], gl * el));
  // a = w_0 / gamma_0 = e_0 / sum;  b_m = w_m - a gamma_m = gamma_m (e_m - e_0) / sum
  const double an = e[0] * inv, gi = gl * inv;
  if constexpr (SI) {
    a = an;
#pragma unroll
    for (int m = 0; m < NM; ++m) b[m] = gi * (e[m + 1] - e[0]);
  } else {
    // linear weights: a = 1, b = 0 exactly
    a = fma(an, P.nonlin, 1.0 - P.nonlin);
    const double gi_n = gi * P.nonlin;
#pragma unroll
    for (int m = 0; m < NM; ++m) b[m] = gi_n * (e[m + 1] - e[0]);
  }
}

// ---------------------------------------------------------------------------
// 1D: one scalar reconstruction
// ---------------------------------------------------------------------------
// Input: u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1} (FP64).  Output: combined
// polynomial coefficients C0..C4 in xi (in TR) and the modified moment.
template <class TR>
struct Poly1 {
  TR c[5];
};

__device__ __forceinline__ void p0_coeffs_1d(double um, double u0, double up, double vm, double vp,
                                             double (&c)[5]) {
  const double su = um + up, du = up - um, sv = vm + vp, dv = vp - vm;
  c[0] = (-43.0 / 384.0) * su + (235.0 / 192.0) * u0 + (27.0 / 64.0) * dv;
  c[1] = (63.0 / 76.0) * du - (75.0 / 19.0) * sv;
  c[2] = (23.0 / 16.0) * su - (23.0 / 8.0) * u0 - (45.0 / 8.0) * dv;
  c[3] = (-5.0 / 19.0) * du + (60.0 / 19.0) * sv;
  c[4] = (-5.0 / 8.0) * su + (5.0 / 4.0) * u0 + (15.0 / 4.0) * dv;
}

__device__ __forceinline__ double beta0_1d(const double (&c)[5]) {
  const double t1 = c[1] + 0.25 * c[3];
  const double t2 = c[2] + (63.0 / 130.0) * c[4];
  return t1 * t1 + (13.0 / 3.0) * t2 * t2 + (781.0 / 20.0) * c[3] * c[3] +
         (1421461.0 / 2275.0) * c[4] * c[4];
}

// c: p0 coefficients; slopes s1 = u_i - u_{i-1}, s2 = u_{i+1} - u_i; u0 = u_i.
// |u| values for u_ave are passed separately (characteristic or scalar).
template <class TR>
__device__ __forceinline__ void hweno_1d(const SchemeParams& P, const double (&c)[5], double u0,
                                         double s1, double s2, double aum, double au0, double aup,
                                         TR (&C)[5]) {
  double beta[3] = {beta0_1d(c), s1 * s1, s2 * s2};
  const double ua = (aum + au0 + aup) * (1.0 / 3.0);
  double a, b[2];
  combine_factors<2, false, TR, true>(P, beta, ua * ua, a, b);
  C[0] = (TR)(a * c[0] + (b[0] + b[1]) * u0);
  C[1] = (TR)(a * c[1] + b[0] * s1 + b[1] * s2);
  C[2] = (TR)(a * c[2]);
  C[3] = (TR)(a * c[3]);
  C[4] = (TR)(a * c[4]);
}

// values at xi = -1/2, -sqrt5/10, +sqrt5/10, +1/2 and the x-moment
template <class TR>
__device__ __forceinline__ void eval_1d(const TR (&C)[5], TR (&pt)[4], TR& mom) {
  const TR h = (TR)0.5, s = (TR)GL4S;
  const TR Eh = C[0] + h * h * (C[2] + h * h * C[4]);
  const TR Oh = h * (C[1] + h * h * C[3]);
  const TR Es = C[0] + s * s * (C[2] + s * s * C[4]);
  const TR Os = s * (C[1] + s * s * C[3]);
  pt[0] = Eh - Oh;
  pt[1] = Es - Os;
  pt[2] = Es + Os;
  pt[3] = Eh + Oh;
  mom = C[1] * (TR)(1.0 / 12.0) + C[3] * (TR)(1.0 / 80.0);
}

// ---------------------------------------------------------------------------
// 2D: stencil data and one scalar reconstruction
// ---------------------------------------------------------------------------
// Stencil layout: u[0..8] = cells 1..9 (label = 5 + a + 3b for offset (a, b)),
// v[0..3] = v at cells 2, 4, 6, 8, w[0..3] = w at cells 2, 4, 6, 8.
struct Sten2 {
  double u[9];
  double v[4];
  double w[4];
};

__device__ __forceinline__ void p0_coeffs_2d(const Sten2& s, double (&c)[15]) {
  const double u1 = s.u[0], u2 = s.u[1], u3 = s.u[2], u4 = s.u[3], u5 = s.u[4], u6 = s.u[5],
               u7 = s.u[6], u8 = s.u[7], u9 = s.u[8];
  const double v2 = s.v[0], v4 = s.v[1], v6 = s.v[2], v8 = s.v[3];
  const double w2 = s.w[0], w4 = s.w[1], w6 = s.w[2], w8 = s.w[3];
  const double corner = u1 + u3 + u7 + u9;
  const double ux = -u1 + u3 - u7 + u9;  // x-odd corner combination
  const double uy = -u1 - u3 + u7 + u9;  // y-odd corner combination
  const double uxy = u1 - u3 - u7 + u9;  // xy-odd corner combination
  c[0] = (1.0 / 576.0) * corner - (133.0 / 1152.0) * (u2 + u4 + u6 + u8) + (419.0 / 288.0) * u5 +
         (27.0 / 64.0) * (v6 - v4) + (27.0 / 64.0) * (w8 - w2);
  c[1] = (-1.0 / 48.0) * ux + (397.0 / 456.0) * (u6 - u4) - (75.0 / 19.0) * (v4 + v6);
  c[2] = (-1.0 / 48.0) * uy + (397.0 / 456.0) * (u8 - u2) - (75.0 / 19.0) * (w2 + w8);
  c[3] = (-1.0 / 48.0) * corner + (1.0 / 24.0) * (u2 + u8) + (71.0 / 48.0) * (u4 + u6) -
         (71.0 / 24.0) * u5 + (45.0 / 8.0) * (v4 - v6);
  c[4] = (-7.0 / 22.0) * uxy + (75.0 / 11.0) * (v8 - v2) + (75.0 / 11.0) * (w6 - w4);
  c[5] = (-1.0 / 48.0) * corner + (71.0 / 48.0) * (u2 + u8) + (1.0 / 24.0) * (u4 + u6) -
         (71.0 / 24.0) * u5 + (45.0 / 8.0) * (w2 - w8);
  c[6] = (5.0 / 19.0) * (u4 - u6) + (60.0 / 19.0) * (v4 + v6);
  c[7] = 0.25 * uy + 0.5 * (u2 - u8);
  c[8] = 0.25 * ux + 0.5 * (u4 - u6);
  c[9] = (5.0 / 19.0) * (u2 - u8) + (60.0 / 19.0) * (w2 + w8);
  c[10] = (-5.0 / 8.0) * (u4 + u6) + 1.25 * u5 + (15.0 / 4.0) * (v6 - v4);
  c[11] = (5.0 / 22.0) * uxy + (60.0 / 11.0) * (v2 - v8);
  c[12] = 0.25 * corner - 0.5 * (u2 + u4 + u6 + u8) + u5;
  c[13] = (5.0 / 22.0) * uxy + (60.0 / 11.0) * (w4 - w6);
  c[14] = (-5.0 / 8.0) * (u2 + u8) + 1.25 * u5 + (15.0 / 4.0) * (w8 - w2);
}

__device__ __forceinline__ double sq(double x) { return x * x; }

// printed sum-of-squares form of the smoothness indicator of p0 in 2D
__device__ __forceinline__ double beta0_2d(const double (&c)[15]) {
  double b = 0.5 * (sq(c[1] + 0.5 * c[6]) + sq(c[1] + (1.0 / 6.0) * c[8]) +
                    sq(c[2] + (1.0 / 6.0) * c[7]) + sq(c[2] + 0.5 * c[9]));
  b += (13.0 / 6.0) * (sq(c[3] + (63.0 / 65.0) * c[10]) + sq(c[3] + (1.0 / 6.0) * c[12]) +
                       sq(c[5] + (1.0 / 6.0) * c[12]) + sq(c[5] + (63.0 / 65.0) * c[14]));
  b += (7.0 / 12.0) * (sq(c[4] + (17.0 / 35.0) * c[11]) + sq(c[4] + (17.0 / 35.0) * c[13]));
  b += (3119.0 / 80.0) * sq(c[6] + (5.0 / 9357.0) * c[8]);
  b += (3379.0 / 720.0) * sq(c[7] + (15.0 / 3379.0) * c[9]);
  b += (2634769.0 / 561420.0) * sq(c[8]) + (2634769.0 / 67580.0) * sq(c[9]);
  b += (5676583.0 / 9100.0) * sq(c[10] + (3185.0 / 11353166.0) * c[12]);
  b += (709573.0 / 16800.0) * sq(c[11] + (1155.0 / 709573.0) * c[13]);
  b += (230094013357.0 / 12261419280.0) * sq(c[12] + (2145748374.0 / 230094013357.0) * c[14]);
  b += (31468281769.0 / 745051650.0) * sq(c[13]);
  b += (25118160529227568.0 / 40266452337475.0) * sq(c[14]);
  return b;
}

// Linear polynomials p1..p4 share four one-sided differences:
//   dL = u5 - u4, dR = u6 - u5, dB = u5 - u2, dT = u8 - u5
// p1 = u5 + dL xi + dB eta, p2 = u5 + dR xi + dB eta,
// p3 = u5 + dL xi + dT eta, p4 = u5 + dR xi + dT eta.
// Combined coefficients C from p0 coefficients c, the centre value u5 and
// the differences; |u| of cells 2, 4, 5, 6, 8 for u_ave.
template <class TR, bool SI, bool FOLD = false>
__device__ __forceinline__ void hweno_2d(const SchemeParams& P, const double (&c)[15], double u5,
                                         double dL, double dR, double dB, double dT,
                                         double abs_sum5, TR (&C)[15], double* a_out = nullptr) {
  const double lL = dL * dL, lR = dR * dR, lB = dB * dB, lT = dT * dT;
  double beta[5] = {beta0_2d(c), lL + lB, lR + lB, lL + lT, lR + lT};
  const double ua = abs_sum5 * 0.2;
  double a, b[4];
  combine_factors<4, SI, TR>(P, beta, ua * ua, a, b);
  C[0] = (TR)(a * c[0] + ((b[0] + b[1]) + (b[2] + b[3])) * u5);
  C[1] = (TR)(a * c[1] + (b[0] + b[2]) * dL + (b[1] + b[3]) * dR);
  C[2] = (TR)(a * c[2] + (b[0] + b[1]) * dB + (b[2] + b[3]) * dT);
  if constexpr (FOLD) {
    // C[3..14] left as the p0 coefficients; the caller folds `a` into the
    // factor it multiplies them with
#pragma unroll
    for (int n = 3; n < 15; ++n) C[n] = (TR)c[n];
    *a_out = a;
  } else {
#pragma unroll
    for (int n = 3; n < 15; ++n) C[n] = (TR)(a * c[n]);
  }
}

// moments of the combined polynomial: int C xi, int C eta over the cell
template <class TR>
__device__ __forceinline__ TR qv_2d(const TR (&C)[15]) {
  return C[1] * (TR)(1.0 / 12.0) + C[6] * (TR)(1.0 / 80.0) + C[8] * (TR)(1.0 / 144.0);
}
template <class TR>
__device__ __forceinline__ TR qw_2d(const TR (&C)[15]) {
  return C[2] * (TR)(1.0 / 12.0) + C[9] * (TR)(1.0 / 80.0) + C[7] * (TR)(1.0 / 144.0);
}

// Restriction of the quartic C(xi, eta) to eta = e as a polynomial in xi
// (d0..d4), and to xi = e as a polynomial in eta (dual).
template <class TR>
__device__ __forceinline__ void restrict_eta(const TR (&C)[15], TR e, TR (&d)[5]) {
  d[0] = C[0] + e * (C[2] + e * (C[5] + e * (C[9] + e * C[14])));
  d[1] = C[1] + e * (C[4] + e * (C[8] + e * C[13]));
  d[2] = C[3] + e * (C[7] + e * C[12]);
  d[3] = C[6] + e * C[11];
  d[4] = C[10];
}
template <class TR>
__device__ __forceinline__ void restrict_xi(const TR (&C)[15], TR e, TR (&d)[5]) {
  d[0] = C[0] + e * (C[1] + e * (C[3] + e * (C[6] + e * C[10])));
  d[1] = C[2] + e * (C[4] + e * (C[7] + e * C[11]));
  d[2] = C[5] + e * (C[8] + e * C[12]);
  d[3] = C[9] + e * C[13];
  d[4] = C[14];
}
// The same restrictions to the three Gauss lines g = 0, 1, 2 at -sqrt15/10,
// 0, +sqrt15/10: on the middle line the restriction is a selection of
// coefficients.  (The general form would multiply by zero there, which the
// compiler must keep, since 0 * x is not 0 for every x.)
template <class TR>
__device__ __forceinline__ void restrict_eta_line(const TR (&C)[15], int g, TR (&d)[5]) {
  if (g == 1) {
    d[0] = C[0];
    d[1] = C[1];
    d[2] = C[3];
    d[3] = C[6];
    d[4] = C[10];
  } else {
    restrict_eta<TR>(C, g == 0 ? (TR)-G3S : (TR)G3S, d);
  }
}
template <class TR>
__device__ __forceinline__ void restrict_xi_line(const TR (&C)[15], int g, TR (&d)[5]) {
  if (g == 1) {
    d[0] = C[0];
    d[1] = C[2];
    d[2] = C[5];
    d[3] = C[9];
    d[4] = C[14];
  } else {
    restrict_xi<TR>(C, g == 0 ? (TR)-G3S : (TR)G3S, d);
  }
}
// 1D quartic d at +-1/2 (edges) and +-sqrt15/10, 0 (Gauss points)
template <class TR>
__device__ __forceinline__ void eval5(const TR (&d)[5], TR& em, TR& ep, TR& gm, TR& g0, TR& gp) {
  const TR h2 = (TR)0.25, s = (TR)G3S, s2 = (TR)(G3S * G3S);
  const TR Eh = d[0] + h2 * (d[2] + h2 * d[4]);
  const TR Oh = (TR)0.5 * (d[1] + h2 * d[3]);
  const TR Es = d[0] + s2 * (d[2] + s2 * d[4]);
  const TR Os = s * (d[1] + s2 * d[3]);
  em = Eh - Oh;
  ep = Eh + Oh;
  gm = Es - Os;
  g0 = d[0];
  gp = Es + Os;
}

// ---------------------------------------------------------------------------
// Euler: physical fluxes (ideal gas)
// ---------------------------------------------------------------------------
// physical flux in direction DIR (0 = f, 1 = g) of the conserved state U
template <int EQ, int NC, int DIR, class T>
__device__ __forceinline__ void phys_flux(const SchemeParams& P, const T (&U)[NC], T (&F)[NC]) {
  if constexpr (EQ == EQ_ADVECTION) {
    F[0] = (T)(DIR == 0 ? P.adv_x : P.adv_y) * U[0];
  } else if constexpr (EQ == EQ_BURGERS) {
    F[0] = (T)0.5 * U[0] * U[0];
  } else if constexpr (NC == 3) {
    const T gm1 = (T)(P.gas_gamma - 1.0);
    const T u = U[1] * rcp_nr(U[0]);
    const T p = gm1 * (U[2] - (T)0.5 * U[1] * u);
    F[0] = U[1];
    F[1] = U[1] * u + p;
    F[2] = u * (U[2] + p);
  } else {
    const T gm1 = (T)(P.gas_gamma - 1.0);
    const T rinv = rcp_nr(U[0]);
    const T u = U[1] * rinv, v = U[2] * rinv;
    const T p = gm1 * (U[3] - (T)0.5 * (U[1] * u + U[2] * v));
    if constexpr (DIR == 0) {
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
}

// Twice the Lax-Friedrichs flux: F(u-) + F(u+) - alpha (u+ - u-).  The
// callers fold the factor 1/2 into their quadrature weights (exactly: a
// power of two).
template <int EQ, int NC, int DIR, class T>
__device__ __forceinline__ void lf_flux2(const SchemeParams& P, const T (&um)[NC], const T (&up)[NC],
                                         T alpha, T (&fh2)[NC]) {
  T fm[NC], fp[NC];
  phys_flux<EQ, NC, DIR, T>(P, um, fm);
  phys_flux<EQ, NC, DIR, T>(P, up, fp);
#pragma unroll
  for (int k = 0; k < NC; ++k) fh2[k] = fm[k] + fp[k] - alpha * (up[k] - um[k]);
}

// wave speeds |f'(u)| (x) and |g'(u)| (y) of a cell average, and validity
// Physical-state check without the wave speeds: finite values and, for
// Euler, rho > 0 and p > 0, with p > 0 tested as rho E - |m|^2 / 2 > 0 (the
// same condition for rho > 0, free of the division and square root).
template <int EQ, int NC>
__device__ __forceinline__ bool physical_state(const double (&U)[NC]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NC; ++k) ok = ok && isfinite(U[k]);
  if constexpr (EQ == EQ_EULER) {
    const double m2 = U[1] * U[1] + (NC == 4 ? U[2] * U[2] : 0.0);
    ok = ok && U[0] > 0.0 && U[0] * U[NC - 1] - 0.5 * m2 > 0.0;
  }
  return ok;
}

template <int EQ, int NC>
__device__ __forceinline__ bool wave_speeds(const SchemeParams& P, const double (&U)[NC], double& sx,
                                            double& sy) {
  if constexpr (EQ == EQ_ADVECTION) {
    sx = fabs(P.adv_x);
    sy = fabs(P.adv_y);
    return isfinite(U[0]);
  } else if constexpr (EQ == EQ_BURGERS) {
    sx = sy = fabs(U[0]);
    return isfinite(U[0]);
  } else {
    const double rinv = 1.0 / U[0];
    const double u = U[1] * rinv;
    const double v = NC == 4 ? U[2] * rinv : 0.0;
    const double p = (P.gas_gamma - 1.0) * (U[NC - 1] - 0.5 * U[0] * (u * u + v * v));
    const double c = sqrt(P.gas_gamma * p * rinv);
    sx = fabs(u) + c;
    sy = fabs(v) + c;
    bool ok = U[0] > 0.0 && p > 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) ok = ok && isfinite(U[k]);
    return ok;
  }
}

// Neighbour exchange across the 64 lanes of a wave with DPP wave shifts:
// from_prev(x) on lane i returns x of lane i-1, from_next(x) returns x of lane
// i+1 (lane 0 / lane 63 receive their own value; callers never use it).
__device__ __forceinline__ float from_prev(float x) {
  const int v = __float_as_int(x);
  return __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_next(float x) {
  const int v = __float_as_int(x);
  return __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_prev(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}
__device__ __forceinline__ double from_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}

// wave-wide max of a non-negative double (64 lanes)
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// atomic max for non-negative doubles through their IEEE bit patterns
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

}  // namespace hwenou
