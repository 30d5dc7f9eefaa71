// One fused HWENO-U Runge-Kutta stage in 1D (Section 2.1): reconstruction
// (Steps 1-3), moment modification, Lax-Friedrichs fluxes, the semi-discrete
// right-hand sides of Eq. (2.3) and the modified SSP-RK3 combination of
// Eq. (2.13), for scalar laws and the Euler equations.
//
// Mapping: one wave per 62-cell tile.  Lane l reconstructs cell start-1+l;
// lanes 1..62 own the output cells, lanes 0 and 63 only supply the interface
// values of the neighbouring cells.  Interface values and fluxes move between
// lanes with cross-lane shuffles, so no LDS and no barrier is used.  Every
// interface flux is evaluated once, by the lane on its right, and handed to
// the lane on its left, which keeps the update conservative to round-off.
// Waves take contiguous runs of tiles from a per-wave work list (a persistent
// launch), so one launch advances any number of instances of uneven size.
#include <algorithm>

#include "hwenou_internal.hpp"

namespace hwenou {

// A read of data that no kernel writes while a stage kernel runs (the work
// list, the instance records, the done flags, alpha and dt), through the
// constant address space and word by word, so that at a wave-uniform address
// it becomes a scalar load, which does not wait behind the wave's vector
// memory traffic.
template <class T>
__device__ __forceinline__ T load_invariant(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "records of whole 32-bit words");
  using Word = const __attribute__((address_space(4))) unsigned;
  Word* q = (Word*)p;
  unsigned v[sizeof(T) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) v[k] = q[k];
  T r;
  __builtin_memcpy(&r, v, sizeof(T));
  return r;
}

// The boundary rule of bc_index (periodic wrap, transmissive copy, mirror
// image at a reflective wall) as selects, so that the lanes of a tile form
// their source cells without branching on their own indices.
__device__ __forceinline__ int source_cell(int i, int n, int bc_lo, int bc_hi, bool& mirrored) {
  const bool lo = i < 0, out = lo || i >= n;
  const int bc = lo ? bc_lo : bc_hi;
  const int wrap = lo ? i + n : i - n;
  const int mirror = lo ? -1 - i : 2 * n - 1 - i;
  const int edge = lo ? 0 : n - 1;
  mirrored = out && bc == BC_REFLECTIVE;
  const int j = bc == BC_PERIODIC ? wrap : (bc == BC_REFLECTIVE ? mirror : edge);
  return out ? j : i;
}

// Resident waves per SIMD the compiler must allow: the kernel is latency-
// bound, and the mixed characteristic Euler kernel and both component-wise
// Euler kernels fit 4 waves per SIMD (128 registers) without spilling; the
// FP64 characteristic kernel needs more (3 waves) and the scalar laws use far
// fewer, so those keep the compiler's choice.
template <int EQ, bool CHAR, class TR>
constexpr int min_waves_1d() {
  return (EQ == EQ_EULER && (!CHAR || sizeof(TR) == 4)) ? 4 : 1;
}

// ST: the Runge-Kutta stage (0, 1, 2), compiled in like the coefficients.
template <int EQ, bool CHAR, int ST, class TR, class TM>
__global__ __launch_bounds__(256, (min_waves_1d<EQ, CHAR, TR>())) void stage1d_kernel(
    const StageArgs<TM> A) {
  constexpr int NC = EQ == EQ_EULER ? 3 : 1;
  const int lane = threadIdx.x & 63;
  // The wave index is uniform across the wave; saying so lets the compiler
  // read the work list, the instance record, the done flag, alpha and dt with
  // scalar loads (which do not wait behind the wave's vector memory traffic)
  // instead of per-lane vector loads.
  const int w =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (w >= A.n_waves) return;
  const SchemeParams& P = A.P;
  // Runge-Kutta combination out = ra * base + rb * (in + dt F)
  constexpr double ra = ST == 0 ? 0.0 : (ST == 1 ? 0.75 : 1.0 / 3.0);
  constexpr double rb = ST == 0 ? 1.0 : (ST == 1 ? 0.25 : 2.0 / 3.0);
  const long long plane = A.plane;

  const int it_end = load_invariant(A.work_ptr + w + 1);
  for (int it = load_invariant(A.work_ptr + w); it < it_end; ++it) {
    const WorkItem wk = load_invariant(A.work + it);
    // the instance's records are read together, before the done flag is
    // tested, so that they arrive in one round trip
    const bool done = A.done != nullptr && load_invariant(A.done + wk.inst);
    const InstDev I = load_invariant(A.inst + wk.inst);
    const double alpha_in = load_invariant(A.alpha + 2 * wk.inst);
    const double dt = load_invariant(A.dt + wk.inst);
    if (done) continue;
    const int n = I.nx;
    int i = wk.a - 1 + lane;
    // lanes past the right ring lane (i = n) take i = n + 1: the ring lane reads
    // its right neighbour from the next lane; lanes further right are unused
    if (i > n + 1) i = n + 1;
    const bool owner = lane >= 1 && lane <= kStripWidth && i < n;
    bool mir_m, mir_c, mir_p;  // mirror images at reflective walls
    const int im = source_cell(i - 1, n, I.bc[0], I.bc[1], mir_m);
    const int ic = source_cell(i, n, I.bc[0], I.bc[1], mir_c);
    const int ip = source_cell(i + 1, n, I.bc[0], I.bc[1], mir_p);
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
      if (ST != 0 && owner) {
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
      // Characteristic fields of f' at the cell average: left rows
      //   l_0 = (b2 + u/c, -(b1 u + 1/c), b1) / 2,  l_1 = (1 - b2, b1 u, -b1),
      //   l_2 = (b2 - u/c, -(b1 u - 1/c), b1) / 2,
      // right columns r_0 = (1, u - c, H - u c), r_1 = (1, u, u^2/2),
      // r_2 = (1, u + c, H + u c), with b1 = (gamma - 1)/c^2, b2 = b1 u^2/2.
      // The point values and moment P_K of the fields map back as
      //   rho = S + P_1,  m = u rho + c D,  E = H S + u c D + u^2/2 P_1,
      // with S = P_0 + P_2 and D = P_2 - P_0 (in FP64), so no 3x3 matrix is
      // kept and fewer values are live while the fields are reconstructed.
      const double gm1 = P.gas_gamma - 1.0;
      const double rinv = rcp_w<TR>(Uc[0]);
      const double u = Uc[1] * rinv;
      const double pr = gm1 * (Uc[2] - 0.5 * Uc[1] * u);
      const double c2 = (gm1 + 1.0) * pr * rinv;
      const double ci = rsq_w<TR>(c2);
      const double c = c2 * ci;
      const double H = (Uc[2] + pr) * rinv;
      const double b1 = gm1 * (ci * ci);
      const double b2 = 0.5 * b1 * u * u;
      // one field: project with row (l0, l1, l2), reconstruct, evaluate
      auto field = [&](double l0, double l1, double l2, double (&q)[5]) {
        const double wm = l0 * Um[0] + l1 * Um[1] + l2 * Um[2];
        const double wc = l0 * Uc[0] + l1 * Uc[1] + l2 * Uc[2];
        const double wp = l0 * Up[0] + l1 * Up[1] + l2 * Up[2];
        const double vvm = l0 * Vm[0] + l1 * Vm[1] + l2 * Vm[2];
        const double vvp = l0 * Vp[0] + l1 * Vp[1] + l2 * Vp[2];
        double cf[5];
        p0_coeffs_1d(wm, wc, wp, vvm, vvp, cf);
        TR C[5], pts[4], qm;
        hweno_1d<TR>(P, cf, wc, wc - wm, wp - wc, fabs(wm), fabs(wc), fabs(wp), C);
        eval_1d<TR>(C, pts, qm);
#pragma unroll
        for (int g = 0; g < 4; ++g) q[g] = (double)pts[g];
        q[4] = (double)qm;
      };
      double S[5], D[5], Q[5];  // q[0..3] point values, q[4] the moment
      field(0.5 * (b2 + u * ci), -0.5 * (b1 * u + ci), 0.5 * b1, Q);
      field(0.5 * (b2 - u * ci), -0.5 * (b1 * u - ci), 0.5 * b1, S);
#pragma unroll
      for (int g = 0; g < 5; ++g) {
        D[g] = S[g] - Q[g];
        S[g] = S[g] + Q[g];
      }
      field(1.0 - b2, b1 * u, -b1, Q);
#pragma unroll
      for (int g = 0; g < 5; ++g) {
        const double rho = S[g] + Q[g];
        const TR mom = (TR)(u * rho + c * D[g]);
        const TR en = (TR)(H * S[g] + (u * c) * D[g] + (0.5 * u * u) * Q[g]);
        if (g < 4) {
          pt[g][0] = (TR)rho;
          pt[g][1] = mom;
          pt[g][2] = en;
        } else {
          vh[0] = (TR)rho;
          vh[1] = mom;
          vh[2] = en;
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
    const TR alpha = (TR)alpha_in;
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
    const double idx = 1.0 / I.dx;
    double Uo[NC];
    if (owner) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const double F1 = -((double)fr[k] - (double)fl[k]) * (0.5 * idx);
        const TR F2 = -(fl[k] + fr[k]) * (TR)(0.25 * idx) + vol[k] * (TR)idx;
        const double ub = ST == 0 ? 0.0 : Ub[k];
        const double un = ra * ub + rb * (Uc[k] + dt * F1);
        TR mn;
        if (ST == 0) {
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
      if (ST == 2 && A.alpha_next != nullptr)  // the wave speeds feed the next step's alpha
        ok = wave_speeds<EQ, NC>(P, Uo, sx, sy);
      else
        ok = physical_state<EQ, NC>(Uo);
    }
    if (!ok) atomicOr(&A.status[wk.inst], 1);
    if (ST == 2 && A.alpha_next != nullptr) {
      const double mx = wave_max(owner ? sx : 0.0);
      if (lane == 0) atomic_max_nonneg(A.alpha_next + alpha_slot(wk.inst, w, A.alpha_slots), mx);
    }
  }
}

template <int EQ, bool CHAR, class TR, class TM>
static hipError_t launch(const void* args, int blocks, int threads, hipStream_t s) {
  const auto& a = *static_cast<const StageArgs<TM>*>(args);
  switch (a.stage) {
    case 0:
      hipLaunchKernelGGL((stage1d_kernel<EQ, CHAR, 0, TR, TM>), dim3(blocks), dim3(threads), 0, s,
                         a);
      break;
    case 1:
      hipLaunchKernelGGL((stage1d_kernel<EQ, CHAR, 1, TR, TM>), dim3(blocks), dim3(threads), 0, s,
                         a);
      break;
    default:
      hipLaunchKernelGGL((stage1d_kernel<EQ, CHAR, 2, TR, TM>), dim3(blocks), dim3(threads), 0, s,
                         a);
  }
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

template <int EQ, bool CHAR, int ST, class TR, class TM>
static int occupancy_st(int threads) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, stage1d_kernel<EQ, CHAR, ST, TR, TM>,
                                                   threads, 0) != hipSuccess)
    return 0;
  return blocks;
}

// resident blocks per CU common to the three stage kernels
template <int EQ, bool CHAR, class TR, class TM>
static int occupancy(int threads) {
  return std::min(occupancy_st<EQ, CHAR, 0, TR, TM>(threads),
                  std::min(occupancy_st<EQ, CHAR, 1, TR, TM>(threads),
                           occupancy_st<EQ, CHAR, 2, TR, TM>(threads)));
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
