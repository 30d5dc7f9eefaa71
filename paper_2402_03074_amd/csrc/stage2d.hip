// One fused HWENO-U Runge-Kutta stage in 2D (Section 2.2): the true-2D
// quartic reconstruction on the 3x3 stencil (Step 1), smoothness indicators
// and scale-invariant weights (Steps 2-3), the modified moments v^, w^, the
// 21 point values, Lax-Friedrichs fluxes at the 3 Gauss points of every
// edge, the right-hand sides F1, F2, F3 and the modified SSP-RK3 update.
//
// Euler: the reconstruction runs on local characteristic variables in two
// direction-split sweeps.  The x-sweep projects with the eigenvectors of f'
// at the cell average and yields the x-edge values, the interior values used
// for f, and v^; the y-sweep does the same with g' for the y-edges, g and
// w^.  Because the reconstruction is linear in the data, the p0 coefficients
// are formed once per conserved component and projected per sweep.
// Scalar laws (and component-wise Euler) use one reconstruction for both.
//
// Mapping: a wave marches a strip of 62 output columns upward, one row per
// step; lane l holds column strip*62 - 1 + l (lanes 0 and 63 supply the
// neighbour columns' x-edge values).  x-interface values and fluxes move
// between lanes by shuffles; the y-edge values of the previous row and the
// partially accumulated right-hand side of that row stay in registers, so
// each y-flux is evaluated once and each row is written once.  A row's stage
// output is stored when the row above has supplied its upper y-flux.  Waves
// take balanced runs of (strip, rows) from a per-wave work list, so one
// persistent launch covers one large grid or many instances of uneven size.
#include "hwenou_internal.hpp"

namespace hwenou {

// load the 3x3 stencil of cell (i, j) (wrapped/clamped indices)
template <int NC, class TM>
__device__ __forceinline__ void load_stencil(const StageArgs<TM>& A, const InstDev& I, int i, int j,
                                             Sten2 (&S)[NC]) {
  const int nx = I.nx, ny = I.ny;
  int xi[3], yj[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xi[d] = wrap_index(i + d - 1, nx, I.bc[0], I.bc[1]);
    yj[d] = wrap_index(j + d - 1, ny, I.bc[2], I.bc[3]);
  }
  const long long plane = A.plane;
  const double* u = A.u_in + I.offset;
  const TM* v = A.m_in + I.offset;
  const TM* w = A.m_in + (long long)NC * plane + I.offset;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) S[k].u[a + 3 * b] = u[k * plane + (long long)yj[b] * nx + xi[a]];
    // cells 2, 4, 6, 8 = offsets (0,-1), (-1,0), (1,0), (0,1)
    const long long c2 = (long long)yj[0] * nx + xi[1], c4 = (long long)yj[1] * nx + xi[0];
    const long long c6 = (long long)yj[1] * nx + xi[2], c8 = (long long)yj[2] * nx + xi[1];
    S[k].v[0] = (double)v[k * plane + c2];
    S[k].v[1] = (double)v[k * plane + c4];
    S[k].v[2] = (double)v[k * plane + c6];
    S[k].v[3] = (double)v[k * plane + c8];
    S[k].w[0] = (double)w[k * plane + c2];
    S[k].w[1] = (double)w[k * plane + c4];
    S[k].w[2] = (double)w[k * plane + c6];
    S[k].w[3] = (double)w[k * plane + c8];
  }
}

// Outputs of one cell's reconstruction used by the fluxes and the RHS.
template <int NC, class TR>
struct CellRecon {
  TR xm[3][NC], xp[3][NC];  // u at (-1/2, eta_G), (+1/2, eta_G)
  TR ym[3][NC], yp[3][NC];  // u at (xi_G, -1/2), (xi_G, +1/2)
  TR volf[NC], volg[NC];    // sum_GH w_G w_H f / g at the interior Gauss points
  TR vh[NC], wh[NC];        // modified moments
  double u5[NC];            // cell average (stage input)
};

__device__ __forceinline__ double g3w(int g) { return g == 1 ? G3W1 : G3W0; }

// evaluate the x-sweep outputs (x-edges, interior f, v^) from conserved-space
// combined coefficients Cc[m][15]
template <int EQ, int NC, class TR>
__device__ __forceinline__ void eval_x_sweep(const SchemeParams& P, const TR (&Cc)[NC][15],
                                             CellRecon<NC, TR>& R, bool also_y) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    R.volf[k] = (TR)0;
    if (also_y) R.volg[k] = (TR)0;
  }
#pragma unroll
  for (int H = 0; H < 3; ++H) {
    const TR e = (TR)(H == 0 ? -G3S : (H == 1 ? 0.0 : G3S));
    TR in[3][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      TR d[5];
      restrict_eta<TR>(Cc[k], e, d);
      TR em, ep, gm, g0, gp;
      eval5<TR>(d, em, ep, gm, g0, gp);
      R.xm[H][k] = em;
      R.xp[H][k] = ep;
      in[0][k] = gm;
      in[1][k] = g0;
      in[2][k] = gp;
    }
#pragma unroll
    for (int G = 0; G < 3; ++G) {
      TR f[NC];
      phys_flux<EQ, NC, 0, TR>(P, in[G], f);
      const TR wgt = (TR)(g3w(G) * g3w(H));
#pragma unroll
      for (int k = 0; k < NC; ++k) R.volf[k] += wgt * f[k];
      if (also_y) {
        TR g[NC];
        phys_flux<EQ, NC, 1, TR>(P, in[G], g);
#pragma unroll
        for (int k = 0; k < NC; ++k) R.volg[k] += wgt * g[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) R.vh[k] = qv_2d<TR>(Cc[k]);
}

// y-sweep outputs (y-edges, interior g, w^)
template <int EQ, int NC, class TR>
__device__ __forceinline__ void eval_y_sweep(const SchemeParams& P, const TR (&Cc)[NC][15],
                                             CellRecon<NC, TR>& R, bool interior) {
  if (interior) {
#pragma unroll
    for (int k = 0; k < NC; ++k) R.volg[k] = (TR)0;
  }
#pragma unroll
  for (int G = 0; G < 3; ++G) {
    const TR e = (TR)(G == 0 ? -G3S : (G == 1 ? 0.0 : G3S));
    TR in[3][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      TR d[5];
      restrict_xi<TR>(Cc[k], e, d);
      TR em, ep, gm, g0, gp;
      eval5<TR>(d, em, ep, gm, g0, gp);
      R.ym[G][k] = em;
      R.yp[G][k] = ep;
      in[0][k] = gm;
      in[1][k] = g0;
      in[2][k] = gp;
    }
    if (interior) {
#pragma unroll
      for (int H = 0; H < 3; ++H) {
        TR g[NC];
        phys_flux<EQ, NC, 1, TR>(P, in[H], g);
        const TR wgt = (TR)(g3w(G) * g3w(H));
#pragma unroll
        for (int k = 0; k < NC; ++k) R.volg[k] += wgt * g[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) R.wh[k] = qw_2d<TR>(Cc[k]);
}

// characteristic sweep: project conserved p0 coefficients with L, weight
// per characteristic field, back-project the combined polynomial with R
template <int DIR, class TR>
__device__ __forceinline__ void char_sweep(const SchemeParams& P, const double (&c)[4][15],
                                           const double (&u5)[4], const double (&dL)[4],
                                           const double (&dR)[4], const double (&dB)[4],
                                           const double (&dT)[4], TR (&Cc)[4][15]) {
  double L[4][4], R[4][4];
  euler_eig<4, DIR>(P.gas_gamma - 1.0, u5, L, R);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < 15; ++n) Cc[k][n] = (TR)0;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    double cc[15];
#pragma unroll
    for (int n = 0; n < 15; ++n) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += L[ch][k] * c[k][n];
      cc[n] = s;
    }
    double w5 = 0, wL = 0, wR = 0, wB = 0, wT = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w5 += L[ch][k] * u5[k];
      wL += L[ch][k] * dL[k];
      wR += L[ch][k] * dR[k];
      wB += L[ch][k] * dB[k];
      wT += L[ch][k] * dT[k];
    }
    const double asum = fabs(w5 - wB) + fabs(w5 - wL) + fabs(w5) + fabs(w5 + wR) + fabs(w5 + wT);
    TR C[15];
    hweno_2d<TR>(P, cc, w5, wL, wR, wB, wT, asum, C);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const TR r = (TR)R[k][ch];
#pragma unroll
      for (int n = 0; n < 15; ++n) Cc[k][n] += r * C[n];
    }
  }
}

// Reconstruct cell (i, j).  need_x: x-edge values, f and v^ are needed.
template <int EQ, bool CHAR, class TR, class TM>
__device__ __forceinline__ void reconstruct_cell(const StageArgs<TM>& A, const InstDev& I, int i,
                                                 int j, bool need_x,
                                                 CellRecon<(EQ == EQ_EULER ? 4 : 1), TR>& R) {
  constexpr int NC = EQ == EQ_EULER ? 4 : 1;
  const SchemeParams& P = A.P;
  Sten2 S[NC];
  load_stencil<NC, TM>(A, I, i, j, S);
  double c[NC][15], u5[NC], dL[NC], dR[NC], dB[NC], dT[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    p0_coeffs_2d(S[k], c[k]);
    u5[k] = S[k].u[4];
    dL[k] = S[k].u[4] - S[k].u[3];
    dR[k] = S[k].u[5] - S[k].u[4];
    dB[k] = S[k].u[4] - S[k].u[1];
    dT[k] = S[k].u[7] - S[k].u[4];
    R.u5[k] = u5[k];
  }
  if constexpr (EQ == EQ_EULER && CHAR) {
    TR Cc[4][15];
    if (need_x) {
      char_sweep<0, TR>(P, c, u5, dL, dR, dB, dT, Cc);
      eval_x_sweep<EQ, 4, TR>(P, Cc, R, false);
    }
    char_sweep<1, TR>(P, c, u5, dL, dR, dB, dT, Cc);
    eval_y_sweep<EQ, 4, TR>(P, Cc, R, need_x);
  } else {
    TR Cc[NC][15];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double asum = fabs(S[k].u[1]) + fabs(S[k].u[3]) + fabs(S[k].u[4]) + fabs(S[k].u[5]) +
                          fabs(S[k].u[7]);
      hweno_2d<TR>(P, c[k], u5[k], dL[k], dR[k], dB[k], dT[k], asum, Cc[k]);
    }
    // one reconstruction: the interior values serve both f and g
    if (need_x) eval_x_sweep<EQ, NC, TR>(P, Cc, R, true);
    eval_y_sweep<EQ, NC, TR>(P, Cc, R, false);
  }
}

template <int EQ, bool CHAR, class TR, class TM>
__global__ __launch_bounds__(64) void stage2d_kernel(const StageArgs<TM> A) {
  constexpr int NC = EQ == EQ_EULER ? 4 : 1;
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x;
  if (w >= A.n_waves) return;
  const SchemeParams& P = A.P;
  double ra = 0.0, rb = 1.0;
  if (A.stage == 1) { ra = 0.75; rb = 0.25; }
  if (A.stage == 2) { ra = 1.0 / 3.0; rb = 2.0 / 3.0; }
  const long long plane = A.plane;
  const TR gxs[3] = {(TR)(-G3S), (TR)0, (TR)G3S};

  for (int it = A.work_ptr[w]; it < A.work_ptr[w + 1]; ++it) {
    const WorkItem wk = A.work[it];
    if (A.done != nullptr && A.done[wk.inst]) continue;
    const InstDev I = A.inst[wk.inst];
    int i = wk.a * kStripWidth - 1 + lane;
    if (i > I.nx) i = I.nx;
    const bool col_owner = lane >= 1 && lane <= kStripWidth && i < I.nx;
    const TR a1 = (TR)A.alpha[2 * wk.inst], a2 = (TR)A.alpha[2 * wk.inst + 1];
    const double dt = A.dt[wk.inst];
    const double idx = 1.0 / I.dx, idy = 1.0 / I.dy;
    const int r0 = wk.b, r1 = wk.c;

    // carried from the row below: its upper y-edge values, its pending RHS,
    // its modified moments and its cell average
    TR yprev[3][NC];
    double F1p[NC];
    TR F2p[NC], F3p[NC], vhp[NC], whp[NC];
    double u5p[NC];
    double amax_x = 0.0, amax_y = 0.0;
    bool ok = true;

    for (int j = r0 - 1; j <= r1; ++j) {
      const bool row_out = j >= r0 && j < r1;
      CellRecon<NC, TR> R;
      reconstruct_cell<EQ, CHAR, TR, TM>(A, I, i, j, row_out, R);

      // y-flux at y_{j-1/2}: u- = row below at eta=+1/2, u+ = this row at -1/2
      TR gb[3][NC];
      if (j >= r0) {
#pragma unroll
        for (int G = 0; G < 3; ++G) lf_flux<EQ, NC, 1, TR>(P, yprev[G], R.ym[G], a2, gb[G]);
      }
      // finish the row below
      if (j - 1 >= r0 && j - 1 < r1) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          TR s = (TR)0, sm = (TR)0;
#pragma unroll
          for (int G = 0; G < 3; ++G) {
            s += (TR)g3w(G) * gb[G][k];
            sm += (TR)g3w(G) * gxs[G] * gb[G][k];
          }
          F1p[k] -= (double)s * idy;
          F2p[k] -= sm * (TR)idy;
          F3p[k] -= s * (TR)(0.5 * idy);
        }
        if (col_owner) {
          const long long o = I.offset + (long long)(j - 1) * I.nx + i;
          double Uo[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            const double ub = A.stage == 0 ? 0.0 : A.u_base[k * plane + o];
            const double un = ra * ub + rb * (u5p[k] + dt * F1p[k]);
            TR vn, wn;
            if (A.stage == 0) {
              A.m_base[k * plane + o] = (TM)vhp[k];
              A.m_base[(NC + k) * plane + o] = (TM)whp[k];
              vn = vhp[k] + (TR)dt * F2p[k];
              wn = whp[k] + (TR)dt * F3p[k];
            } else {
              const TR vb = (TR)A.m_base[k * plane + o];
              const TR wb = (TR)A.m_base[(NC + k) * plane + o];
              vn = (TR)ra * vb + (TR)rb * (vhp[k] + (TR)dt * F2p[k]);
              wn = (TR)ra * wb + (TR)rb * (whp[k] + (TR)dt * F3p[k]);
            }
            A.u_out[k * plane + o] = un;
            A.m_out[k * plane + o] = (TM)vn;
            A.m_out[(NC + k) * plane + o] = (TM)wn;
            Uo[k] = un;
          }
          double sx, sy;
          ok = wave_speeds<EQ, NC>(P, Uo, sx, sy) && ok;
          amax_x = fmax(amax_x, sx);
          amax_y = fmax(amax_y, sy);
        }
      }
      if (row_out) {
        // x-fluxes of this row at the 3 Gauss points of each x-edge
        TR F2x[NC], F3x[NC];
        double F1x[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          F1x[k] = 0.0;
          F2x[k] = (TR)0;
          F3x[k] = (TR)0;
        }
#pragma unroll
        for (int G = 0; G < 3; ++G) {
          TR um[NC], fl[NC], fr[NC];
#pragma unroll
          for (int k = 0; k < NC; ++k) um[k] = __shfl_up(R.xp[G][k], 1, 64);
          lf_flux<EQ, NC, 0, TR>(P, um, R.xm[G], a1, fl);
#pragma unroll
          for (int k = 0; k < NC; ++k) fr[k] = __shfl_down(fl[k], 1, 64);
          const TR wg = (TR)g3w(G);
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            F1x[k] += (double)wg * ((double)fr[k] - (double)fl[k]);
            F2x[k] += wg * (fl[k] + fr[k]);
            F3x[k] += wg * gxs[G] * (fr[k] - fl[k]);
          }
        }
        // pending RHS of this row: x-terms, volume terms, lower y-flux
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          TR s = (TR)0, sm = (TR)0;
#pragma unroll
          for (int G = 0; G < 3; ++G) {
            s += (TR)g3w(G) * gb[G][k];
            sm += (TR)g3w(G) * gxs[G] * gb[G][k];
          }
          F1p[k] = -F1x[k] * idx + (double)s * idy;
          F2p[k] = -F2x[k] * (TR)(0.5 * idx) + R.volf[k] * (TR)idx + sm * (TR)idy;
          F3p[k] = -F3x[k] * (TR)idx + R.volg[k] * (TR)idy - s * (TR)(0.5 * idy);
          vhp[k] = R.vh[k];
          whp[k] = R.wh[k];
          u5p[k] = R.u5[k];
        }
      }
#pragma unroll
      for (int G = 0; G < 3; ++G)
#pragma unroll
        for (int k = 0; k < NC; ++k) yprev[G][k] = R.yp[G][k];
    }
    if (!ok) atomicOr(A.status, 1);
    if (A.alpha_next != nullptr) {
      const double mx = wave_max(amax_x), my = wave_max(amax_y);
      if (lane == 0) {
        atomic_max_nonneg(&A.alpha_next[2 * wk.inst], mx);
        atomic_max_nonneg(&A.alpha_next[2 * wk.inst + 1], my);
      }
    }
  }
}

template <int EQ, bool CHAR, class TR, class TM>
static hipError_t launch(const void* args, int blocks, int threads, hipStream_t s) {
  const auto& a = *static_cast<const StageArgs<TM>*>(args);
  hipLaunchKernelGGL((stage2d_kernel<EQ, CHAR, TR, TM>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stage_2d(int eq, bool char_decomp, bool mixed, const void* args, int blocks,
                           int threads, hipStream_t s) {
  if (mixed) {
    switch (eq) {
      case EQ_ADVECTION: return launch<EQ_ADVECTION, false, float, float>(args, blocks, threads, s);
      case EQ_BURGERS: return launch<EQ_BURGERS, false, float, float>(args, blocks, threads, s);
      default:
        return char_decomp ? launch<EQ_EULER, true, float, float>(args, blocks, threads, s)
                           : launch<EQ_EULER, false, float, float>(args, blocks, threads, s);
    }
  }
  switch (eq) {
    case EQ_ADVECTION: return launch<EQ_ADVECTION, false, double, double>(args, blocks, threads, s);
    case EQ_BURGERS: return launch<EQ_BURGERS, false, double, double>(args, blocks, threads, s);
    default:
      return char_decomp ? launch<EQ_EULER, true, double, double>(args, blocks, threads, s)
                         : launch<EQ_EULER, false, double, double>(args, blocks, threads, s);
  }
}

}  // namespace hwenou
