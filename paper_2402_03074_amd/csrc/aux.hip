// Auxiliary kernels of the time loop: the maximum wave speed
// alpha = max |f'(u)| over the cell averages (Section 2.1, used by the
// Lax-Friedrichs flux and the CFL condition), the per-instance time step
// dt = min(CFL dx / alpha, T - t) in 1D and CFL / (alpha_1/dx + alpha_2/dy)
// in 2D, and the per-step bookkeeping of t, the step count and completion.
// All per-instance state lives on the device so that whole steps can be
// replayed from a captured graph without host synchronisation.
#include "hwenou_internal.hpp"

namespace hwenou {

template <int EQ, int NC>
__global__ __launch_bounds__(256) void max_wavespeed_kernel(const AuxArgs A) {
  const int inst = blockIdx.y;
  const InstDev I = A.inst[inst];
  const long long n = (long long)I.nx * I.ny;
  double mx = 0.0, my = 0.0;
  bool ok = true;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    double U[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) U[k] = A.u[k * A.plane + I.offset + c];
    double sx, sy;
    ok = wave_speeds<EQ, NC>(A.P, U, sx, sy) && ok;
    mx = fmax(mx, sx);
    my = fmax(my, sy);
  }
  if (!ok) atomicOr(&A.status[inst], 1);
  mx = wave_max(mx);
  my = wave_max(my);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(&A.alpha[2 * inst], mx);
    atomic_max_nonneg(&A.alpha[2 * inst + 1], my);
  }
}

__global__ void zero_alpha_kernel(double* alpha, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    alpha[k] = 0.0;
}

hipError_t launch_max_wavespeed(const AuxArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(zero_alpha_kernel, dim3(1), dim3(256), 0, s, a.alpha, 2 * a.n_inst);
  // 64 blocks per instance, grid-stride over its cells
  const dim3 grid(64, a.n_inst);
  if (a.eq == EQ_ADVECTION)
    hipLaunchKernelGGL((max_wavespeed_kernel<EQ_ADVECTION, 1>), grid, dim3(256), 0, s, a);
  else if (a.eq == EQ_BURGERS)
    hipLaunchKernelGGL((max_wavespeed_kernel<EQ_BURGERS, 1>), grid, dim3(256), 0, s, a);
  else if (a.dim == 1)
    hipLaunchKernelGGL((max_wavespeed_kernel<EQ_EULER, 3>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((max_wavespeed_kernel<EQ_EULER, 4>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Time step of instance k for the step that starts at time t after `steps`
// steps, from its wave speeds (ax, ay); marks the instance done when it has
// reached t_final or max_steps, or when a kernel has flagged one of its
// states as non-physical or non-finite (dt = 0 then: the instance stops at
// the step that failed, and its t and step count say where).  The wave
// speeds are reduced with fmax, which drops NaN arguments, so a NaN state is
// caught by the flag, not by alpha.  The caller passes the values it has
// loaded, so that each step's bookkeeping costs one round of loads.  Returns
// whether the instance is done.
__device__ bool set_step(const AuxArgs& A, int k, const InstDev& I, const RunParams& R, bool done,
                         double t, int steps, int status, double ax, double ay) {
  const bool finished = done || steps >= R.max_steps || t >= R.t_final * (1.0 - 1e-14);
  if (finished || status) {
    A.done[k] = 1;
    A.dt[k] = 0.0;
    return true;
  }
  if (A.dim == 1) ay = 0.0;
  if (!isfinite(ax) || !isfinite(ay)) {  // infinite wave speed: stop and report it
    A.done[k] = 1;
    A.dt[k] = 0.0;
    atomicOr(&A.status[k], 1);
    return true;
  }
  double dt;
  if (ax == 0.0 && ay == 0.0)
    dt = R.t_final - t;  // zero wave speed: every flux vanishes, the CFL bound is infinite
  else if (A.dim == 1)
    dt = R.cfl * I.dx / ax;
  else
    dt = R.cfl / (ax / I.dx + ay / I.dy);
  if (t + dt > R.t_final) dt = R.t_final - t;
  A.dt[k] = dt;
  return false;
}

// Before the first step: its time step, and the reset of the wave-speed
// accumulators that the last stage of the step fills.
__global__ __launch_bounds__(256) void dt_kernel(const AuxArgs A) {
  for (int k = threadIdx.x; k < A.n_inst * A.alpha_slots; k += blockDim.x) {
    A.alpha_next[kAlphaStride * k] = 0.0;
    A.alpha_next[kAlphaStride * k + 1] = 0.0;
  }
  for (int k = threadIdx.x; k < A.n_inst; k += blockDim.x)
    set_step(A, k, A.inst[k], *A.run, A.done[k] != 0, A.t[k], A.steps[k], A.status[k],
             A.alpha[2 * k], A.alpha[2 * k + 1]);
}

// End of a step: advance t and the step count, take the new wave speed,
// reset its accumulator, set the next step's time step, and count the
// instances still running (read by the host every few steps).  Everything
// an instance needs is loaded up front, in one round of loads.
__global__ __launch_bounds__(256) void finish_kernel(const AuxArgs A) {
  __shared__ int running;
  if (threadIdx.x == 0) running = 0;
  __syncthreads();
  int mine = 0;
  const RunParams R = *A.run;
  for (int k = threadIdx.x; k < A.n_inst; k += blockDim.x) {
    double* acc = A.alpha_next + alpha_slot(k, 0, A.alpha_slots);
    const bool done = A.done[k] != 0;
    double t = A.t[k];
    const double dt = A.dt[k];
    int steps = A.steps[k];
    const int status = A.status[k];
    const InstDev I = A.inst[k];
    // every slot line of the allocation is loaded at once (in bounds: the
    // array holds kAlphaSlots lines per instance), and those beyond this
    // instance's slots count as zero (the wave speeds are non-negative)
    double sx[kAlphaSlots], sy[kAlphaSlots];
#pragma unroll
    for (int s = 0; s < kAlphaSlots; ++s) {
      sx[s] = acc[kAlphaStride * s];
      sy[s] = acc[kAlphaStride * s + 1];
    }
    double ax, ay;
    if (!done) {
      t += dt;
      steps += 1;
      ax = sx[0];
      ay = sy[0];
#pragma unroll
      for (int s = 1; s < kAlphaSlots; ++s) {
        const bool own = s < A.alpha_slots;
        ax = fmax(ax, own ? sx[s] : 0.0);
        ay = fmax(ay, own ? sy[s] : 0.0);
      }
      A.t[k] = t;
      A.steps[k] = steps;
      A.alpha[2 * k] = ax;
      A.alpha[2 * k + 1] = ay;
    } else {
      ax = ay = 0.0;  // unused: a done instance stays done
    }
#pragma unroll
    for (int s = 0; s < kAlphaSlots; ++s) {
      if (s < A.alpha_slots) {
        acc[kAlphaStride * s] = 0.0;
        acc[kAlphaStride * s + 1] = 0.0;
      }
    }
    if (!set_step(A, k, I, R, done, t, steps, status, ax, ay)) mine = 1;
  }
  if (mine) atomicOr(&running, 1);
  __syncthreads();
  if (threadIdx.x == 0) A.all_done[0] = running ? 0 : 1;
}

hipError_t launch_dt(const AuxArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finish(const AuxArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hwenou
