// Internal interface between the host library (hwenou_api.cpp) and the
// kernel translation units.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hwenou_device.hpp"

namespace hwenou {

// One problem instance as the kernels see it.
struct InstDev {
  int nx, ny;        // cells (ny = 1 in 1D)
  int bc[4];         // x-lo, x-hi, y-lo, y-hi (BC_*)
  double dx, dy;     // mesh sizes
  long long offset;  // first cell of the instance in each component plane
};

// One work item.  1D: (inst, first cell of a 62-cell tile).  2D: (inst,
// strip, first row, end row) -- a strip is 62 output columns marched upward.
struct WorkItem {
  int inst, a, b, c;
};

// Lanes of a wave that produce output; lane 0 and lane 63 only reconstruct
// the neighbouring cells whose interface values the strip needs.
constexpr int kStripWidth = 62;

// The last stage reduces the wave speeds of its output into `slots`
// accumulators per instance (a power of two up to kAlphaSlots; the wave's
// index picks one), so that ~1000 waves ending together on one instance do
// not all serialise their atomics on one address.  Each accumulator (x and y
// wave speed) sits in a 128-byte line of its own (kAlphaStride doubles),
// since the atomics of one line are serialised as well; the finish kernel
// takes the maximum of the slots.  Handles of many instances use fewer slots
// per instance: few waves end on any one instance at a time, and the finish
// kernel's loop over the slots grows with their number.
constexpr int kAlphaSlots = 16;
constexpr int kAlphaStride = 16;
__device__ __host__ __forceinline__ int alpha_slot(int inst, int wave, int slots) {
  return kAlphaStride * (inst * slots + (wave & (slots - 1)));
}

template <class TM>
struct StageArgs {
  SchemeParams P;
  const InstDev* inst;
  const double* dt;     // [n_inst]
  const double* alpha;  // [n_inst][2]
  const int* done;      // [n_inst] or nullptr
  const double* u_in;   // [nc][plane]
  const TM* m_in;       // [dim][nc][plane]
  const double* u_base; // u^n for stages 1, 2
  TM* m_base;           // v^_n (and w^_n): written by stage 0, read by stages 1, 2
  double* u_out;
  TM* m_out;
  double* alpha_next;   // [n_inst][alpha_slots][kAlphaStride] or nullptr: max wave speed of
                        // the output (x, y in the first two doubles of each slot)
  int alpha_slots;      // accumulators per instance (power of two, <= kAlphaSlots)
  int* status;          // [n_inst]: set to 1 on a non-physical or non-finite output
  long long plane;      // cells per component plane
  const WorkItem* work;
  const int* work_ptr;  // wave w handles work[work_ptr[w] .. work_ptr[w+1])
  int n_waves;
  int stage;            // 0, 1, 2
};

// Host helpers shared by the entry points (hwenou_api.hip).
}  // namespace hwenou
struct hwenou_desc;
struct hwenou_inst;
namespace hwenou {
int check_desc(const hwenou_desc* d);                           // HWENOU_OK or an error code
int check_inst(const hwenou_desc* d, const hwenou_inst& inst);  // one instance's own checks
InstDev inst_dev(const hwenou_desc* d, const hwenou_inst& inst);
SchemeParams scheme_params(const hwenou_desc& d);

// kernel launchers (one per translation unit); return hipSuccess or the launch error.
// char_mode (Euler): 0 component-wise, 1 direction-split characteristic, 2 single
// x-projection (the same as 1 in 1D)
hipError_t launch_stage_1d(int eq, int char_mode, bool mixed, const void* args, int blocks,
                           int threads, hipStream_t s);
// scale_invariant: the default weights, compiled into their own 2D kernels
hipError_t launch_stage_2d(int eq, int char_mode, bool mixed, bool scale_invariant,
                           const void* args, int blocks, int threads, hipStream_t s);

// resident blocks per compute unit of a stage kernel at `threads` per block
int occupancy_stage_1d(int eq, int char_mode, bool mixed, int threads);
int occupancy_stage_2d(int eq, int char_mode, bool mixed, bool scale_invariant, int threads);

// Parameters of one hwenou_advance call, read by the time-step kernels from
// device memory so that a captured step graph stays valid across calls.
struct RunParams {
  double cfl, t_final;
  int max_steps;
};

// auxiliary kernels
struct AuxArgs {
  SchemeParams P;
  int eq, dim, n_inst;
  const InstDev* inst;
  long long plane;
  const double* u;       // [nc][plane]
  double* alpha;         // [n_inst][2]
  double* dt;            // [n_inst]
  double* t;             // [n_inst]
  int* steps;            // [n_inst]
  int* done;             // [n_inst]
  int* status;           // [n_inst]: 1 once the instance left the physical states
  double* alpha_next;    // [n_inst][alpha_slots][kAlphaStride]
  int alpha_slots;
  const RunParams* run;  // CFL number, final time, step limit
  int* all_done;         // 1 when every instance is done
};
hipError_t launch_max_wavespeed(const AuxArgs& a, hipStream_t s);
hipError_t launch_dt(const AuxArgs& a, hipStream_t s);
hipError_t launch_finish(const AuxArgs& a, hipStream_t s);

}  // namespace hwenou
