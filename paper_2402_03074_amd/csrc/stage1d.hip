// One fused HWENO-U Runge-Kutta stage in 1D (Section 2.1): reconstruction
// (Steps 1-3), moment modification, Lax-Friedrichs fluxes, the semi-discrete
// right-hand sides of Eq. (2.4) and the modified SSP-RK3 combination of
// Eq. (2.11), for scalar laws and the Euler equations.
//
// Mapping: one wave per 62-cell tile.  Lane l reconstructs cell start-1+l;
// lanes 1..62 own the output cells, lanes 0 and 63 only supply the interface
// values of the neighbouring cells.  Interface values and fluxes move between
// lanes with cross-lane shuffles, so no LDS and no barrier is used.  Every
// interface flux is evaluated once, by the lane on its right, and handed to
// the lane on its left, which keeps the update conservative to round-off.
// Waves take contiguous runs of tiles from a per-wave work list (a persistent
// launch), so one launch advances any number of instances of uneven size.
#include "hwenou_internal.hpp"

namespace hwenou {

template <int EQ, bool CHAR, class TR, class TM>
__global__ __launch_bounds__(256) void stage1d_kernel(const StageArgs<TM> A) {
  constexpr int NC = EQ == EQ_EULER ? 3 : 1;
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= A.n_waves) return;
  const SchemeParams& P = A.P;
  double ra = 0.0, rb = 1.0;  // RK combination out = ra * base + rb * (in + dt F)
  if (A.stage == 1) { ra = 0.75; rb = 0.25; }
  if (A.stage == 2) { ra = 1.0 / 3.0; rb = 2.0 / 3.0; }
  const long long plane = A.plane;

  for (int it = A.work_ptr[w]; it < A.work_ptr[w + 1]; ++it) {
    const WorkItem wk = A.work[it];
    if (A.done != nullptr && A.done[wk.inst]) continue;
    const InstDev I = A.inst[wk.inst];
    const int n = I.nx;
    int i = wk.a - 1 + lane;
    // lanes past the right ring lane (i = n) take i = n + 1: the ring lane reads
    // its right neighbour from the next lane; lanes further right are unused
    if (i > n + 1) i = n + 1;
    const bool owner = lane >= 1 && lane <= kStripWidth && i < n;
    bool mir_m, mir_c, mir_p;  // mirror images at reflective walls
    const int im = bc_index(i - 1, n, I.bc[0], I.bc[1], mir_m);
    const int ic = bc_index(i, n, I.bc[0], I.bc[1], mir_c);
    const int ip = bc_index(i + 1, n, I.bc[0], I.bc[1], mir_p);
    const bool walls = EQ == EQ_EULER && (I.bc[0] == BC_REFLECTIVE || I.bc[1] == BC_REFLECTIVE);
    const double* u = A.u_in + I.offset;
    const TM* m = A.m_in + I.offset;
    const long long o = I.offset + i;

    // Every lane loads its own cell; the neighbours' values come from the
    // adjacent lanes, except at the two ends of the wave, which load them.
    // The Runge-Kutta base of the owned cell is loaded up front as well.
    double Um[NC], Uc[NC], Up[NC], Vm[NC], Vp[NC], Ub[NC];
    TM Mb[NC];
    TM Vc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      Uc[k] = u[k * plane + ic];
      Vc[k] = m[k * plane + ic];
      if (A.stage != 0 && owner) {
        Ub[k] = A.u_base[k * plane + o];
        Mb[k] = A.m_base[k * plane + o];
      }
    }
    const bool edge_lo = lane == 0, edge_hi = lane == 63;
    double Uend[NC];
    TM Vend[NC];
    if (edge_lo || edge_hi) {
      const int ie = edge_lo ? im : ip;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        Uend[k] = u[k * plane + ie];
        Vend[k] = m[k * plane + ie];
      }
    }
    if constexpr (EQ == EQ_EULER) {
      if (walls) {
        if (mir_c) mirror_cell<0, NC>(Uc, reinterpret_cast<TM(*)[NC]>(Vc), 1);
        if ((edge_lo && mir_m) || (edge_hi && mir_p))
          mirror_cell<0, NC>(Uend, reinterpret_cast<TM(*)[NC]>(Vend), 1);
      }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      Um[k] = from_prev(Uc[k]);
      Up[k] = from_next(Uc[k]);
      const TM vm = from_prev(Vc[k]), vp = from_next(Vc[k]);
      Vm[k] = (double)vm;
      Vp[k] = (double)vp;
      if (edge_lo) {
        Um[k] = Uend[k];
        Vm[k] = (double)Vend[k];
      }
      if (edge_hi) {
        Up[k] = Uend[k];
        Vp[k] = (double)Vend[k];
      }
    }

    // ---- reconstruction: point values at the 4 Gauss-Lobatto nodes, v^ ----
    TR pt[4][NC], vh[NC];
    if constexpr (EQ == EQ_EULER && CHAR) {
      double L[3][3], R[3][3];
      euler_eig<3, 0>(P.gas_gamma - 1.0, Uc, L, R);
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int k = 0; k < 3; ++k) pt[g][k] = (TR)0;
#pragma unroll
      for (int k = 0; k < 3; ++k) vh[k] = (TR)0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        double wm = 0, wc = 0, wp = 0, vvm = 0, vvp = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          wm += L[ch][k] * Um[k];
          wc += L[ch][k] * Uc[k];
          wp += L[ch][k] * Up[k];
          vvm += L[ch][k] * Vm[k];
          vvp += L[ch][k] * Vp[k];
        }
        double c[5];
        p0_coeffs_1d(wm, wc, wp, vvm, vvp, c);
        TR C[5];
        hweno_1d<TR>(P, c, wc, wc - wm, wp - wc, fabs(wm), fabs(wc), fabs(wp), C);
        TR q[4], qm;
        eval_1d<TR>(C, q, qm);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const TR r = (TR)R[k][ch];
#pragma unroll
          for (int g = 0; g < 4; ++g) pt[g][k] += r * q[g];
          vh[k] += r * qm;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        double c[5];
        p0_coeffs_1d(Um[k], Uc[k], Up[k], Vm[k], Vp[k], c);
        TR C[5];
        hweno_1d<TR>(P, c, Uc[k], Uc[k] - Um[k], Up[k] - Uc[k], fabs(Um[k]), fabs(Uc[k]),
                     fabs(Up[k]), C);
        TR q[4];
        eval_1d<TR>(C, q, vh[k]);
#pragma unroll
        for (int g = 0; g < 4; ++g) pt[g][k] = q[g];
      }
    }

    // ---- fluxes: the lane on the right of x_{i-1/2} evaluates it ----
    const TR alpha = (TR)A.alpha[2 * wk.inst];
    TR um[NC], up[NC], fl[NC], fr[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      um[k] = from_prev(pt[3][k]);
      up[k] = pt[0][k];
    }
    lf_flux2<EQ, NC, 0, TR>(P, um, up, alpha, fl);  // twice the flux
#pragma unroll
    for (int k = 0; k < NC; ++k) fr[k] = from_next(fl[k]);

    // volume term: Gauss-Lobatto quadrature of f over the cell
    TR vol[NC];
    {
      TR f[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) vol[k] = (TR)0;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        TR q[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) q[k] = pt[g][k];
        phys_flux<EQ, NC, 0, TR>(P, q, f);
        const TR wg = (TR)((g == 0 || g == 3) ? GL4W0 : GL4W1);
#pragma unroll
        for (int k = 0; k < NC; ++k) vol[k] += wg * f[k];
      }
    }

    // ---- semi-discrete RHS and RK combination ----
    const double dt = A.dt[wk.inst];
    const double idx = 1.0 / I.dx;
    double Uo[NC];
    if (owner) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const double F1 = -((double)fr[k] - (double)fl[k]) * (0.5 * idx);
        const TR F2 = -(fl[k] + fr[k]) * (TR)(0.25 * idx) + vol[k] * (TR)idx;
        const double ub = A.stage == 0 ? 0.0 : Ub[k];
        const double un = ra * ub + rb * (Uc[k] + dt * F1);
        TR mn;
        if (A.stage == 0) {
          A.m_base[k * plane + o] = (TM)vh[k];
          mn = vh[k] + (TR)dt * F2;
        } else {
          const TR mb = (TR)Mb[k];
          mn = (TR)ra * mb + (TR)rb * (vh[k] + (TR)dt * F2);
        }
        A.u_out[k * plane + o] = un;
        A.m_out[k * plane + o] = (TM)mn;
        Uo[k] = un;
      }
    }
    double sx = 0.0, sy = 0.0;
    bool ok = true;
    if (owner) {
      if (A.alpha_next != nullptr)  // the wave speeds feed the next step's alpha
        ok = wave_speeds<EQ, NC>(P, Uo, sx, sy);
      else
        ok = physical_state<EQ, NC>(Uo);
    }
    if (!ok) atomicOr(A.status, 1);
    if (A.alpha_next != nullptr) {
      const double mx = wave_max(owner ? sx : 0.0);
      if (lane == 0) atomic_max_nonneg(&A.alpha_next[2 * wk.inst], mx);
    }
  }
}

template <int EQ, bool CHAR, class TR, class TM>
static hipError_t launch(const void* args, int blocks, int threads, hipStream_t s) {
  const auto& a = *static_cast<const StageArgs<TM>*>(args);
  hipLaunchKernelGGL((stage1d_kernel<EQ, CHAR, TR, TM>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stage_1d(int eq, int char_decomp, bool mixed, const void* args, int blocks,
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

template <int EQ, bool CHAR, class TR, class TM>
static int occupancy(int threads) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, stage1d_kernel<EQ, CHAR, TR, TM>, threads, 0) !=
      hipSuccess)
    return 0;
  return blocks;
}

int occupancy_stage_1d(int eq, int char_decomp, bool mixed, int threads) {
  if (mixed) {
    switch (eq) {
      case EQ_ADVECTION: return occupancy<EQ_ADVECTION, false, float, float>(threads);
      case EQ_BURGERS: return occupancy<EQ_BURGERS, false, float, float>(threads);
      default:
        return char_decomp ? occupancy<EQ_EULER, true, float, float>(threads)
                           : occupancy<EQ_EULER, false, float, float>(threads);
    }
  }
  switch (eq) {
    case EQ_ADVECTION: return occupancy<EQ_ADVECTION, false, double, double>(threads);
    case EQ_BURGERS: return occupancy<EQ_BURGERS, false, double, double>(threads);
    default:
      return char_decomp ? occupancy<EQ_EULER, true, double, double>(threads)
                         : occupancy<EQ_EULER, false, double, double>(threads);
  }
}

}  // namespace hwenou
