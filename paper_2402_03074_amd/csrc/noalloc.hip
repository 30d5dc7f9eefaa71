// hwenou_step_noalloc: one modified SSP-RK3 step (Eq. (2.13)) of one
// instance, in place, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  It runs the same stage kernels as hwenou_stage / hwenou_advance;
// what those take from a handle (the stored modified moments of stage 0, two
// stage buffers, the instance record, the work lists, a status word) lives
// here in one file-scope device array of fixed size, `scratch`.
//
// The array's name is only a host-side stand-in for its device address: the
// address is taken once per device with hipGetSymbolAddress (each device holds
// its own copy) and only that pointer is handed to kernels.  Every call on a
// device shares its array: calls that overlap on one device race, and each
// call rebuilds everything it reads from the array (a set-up kernel writes
// the instance record and the work lists and clears the status word).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "../../include/hwenou.h"
#include "hwenou_internal.hpp"

namespace hwenou {
namespace {

constexpr size_t kScratchBytes = HWENOU_NOALLOC_MAX_BYTES;
// the first kHeaderBytes hold the instance record, the status word, the work
// lists; the state buffers follow
constexpr size_t kHeaderBytes = size_t(2) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceInfo {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  int n_cu = 0;
  bool ready = false;
};
DeviceInfo g_dev[kMaxDevices];
std::mutex g_mutex;

// Address of this device's scratch array and its compute-unit count, looked
// up on the first call on the device (with the device current).
int device_info(int dev, DeviceInfo** out) {
  if (dev < 0 || dev >= kMaxDevices) return HWENOU_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mutex);
  DeviceInfo& d = g_dev[dev];
  if (!d.ready) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return HWENOU_EHIP;
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || ncu <= 0) return HWENOU_EHIP;
    d.ptr = static_cast<unsigned char*>(p);
    d.n_cu = ncu;
    d.ready = true;
  }
  *out = &d;
  return HWENOU_OK;
}

// Layout of the header (byte offsets from the start of the array).
constexpr size_t kOffInst = 0;        // InstDev
constexpr size_t kOffStatus = 256;    // int
constexpr size_t kOffPtr = 512;       // int work_ptr[n_waves + 1]

// Writes the instance record, clears the status word, and builds the work
// lists of one instance by formula (the same decomposition as the handle's
// lists: 1D, 62-cell tiles dealt out in contiguous runs; 2D, every strip of
// 62 columns cut into chunks of `per` rows, one chunk per wave).
__global__ void noalloc_setup_kernel(unsigned char* base, InstDev I, int dim, int n_items,
                                     int n_waves, int per, int chunks, size_t off_items,
                                     int use_status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *reinterpret_cast<InstDev*>(base + kOffInst) = I;
    if (use_status) *reinterpret_cast<int*>(base + kOffStatus) = 0;
  }
  int* ptr = reinterpret_cast<int*>(base + kOffPtr);
  WorkItem* items = reinterpret_cast<WorkItem*>(base + off_items);
  if (dim == 1) {
    if (t < n_items) items[t] = {0, t * kStripWidth, 0, 0};
    if (t <= n_waves) ptr[t] = (int)((long long)n_items * t / n_waves);
  } else {
    if (t < n_items) {
      const int s = t / chunks, c = t % chunks;
      const int r0 = c * per, r1 = min(r0 + per, I.ny);
      items[t] = {0, s, r0, r1};
    }
    if (t <= n_waves) ptr[t] = t;  // one item per wave
  }
}

}  // namespace
}  // namespace hwenou

using namespace hwenou;

extern "C" int hwenou_step_noalloc(const hwenou_desc* d, const hwenou_inst* inst, void* stream,
                                   const double* dt_dev, const double* alpha_dev, double* ubar,
                                   void* mom, int* status_dev) {
  if (!d || !inst || !dt_dev || !alpha_dev || !ubar || !mom) return HWENOU_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_inst(d, *inst))) return rc;
  if (inst->offset != 0) return HWENOU_EINVAL;
  const bool mixed = d->precision == HWENOU_MIXED;
  const size_t me = mixed ? 4 : 8;
  const auto al = [](const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; };
  if (!al(ubar, 8) || !al(mom, me) || !al(dt_dev, 8) || !al(alpha_dev, 8) ||
      (status_dev && !al(status_dev, 4)))
    return HWENOU_EINVAL;

  const int dim = d->dim;
  const int nc = d->eq == HWENOU_EQ_EULER ? dim + 2 : 1;
  const int nx = inst->nx, ny = dim == 1 ? 1 : inst->ny;
  const long long cells = (long long)nx * ny;
  // state buffers: stored modified moments, two stage buffers (averages and
  // moments), each 256-byte aligned
  const auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t ub = up((size_t)nc * cells * 8), mb = up((size_t)dim * nc * cells * me);
  if (kHeaderBytes + mb + 2 * (ub + mb) > kScratchBytes) return HWENOU_ESCRATCH;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return HWENOU_EHIP;
  DeviceInfo* di = nullptr;
  if ((rc = device_info(dev, &di))) return rc;

  const int chr = d->eq == HWENOU_EQ_EULER ? d->char_decomp : 0;
  const bool si = d->weights == HWENOU_W_SCALE_INVARIANT;
  int wpc = dim == 1 ? 4 * occupancy_stage_1d(d->eq, chr, mixed, 256)
                     : occupancy_stage_2d(d->eq, chr, mixed, si, 64);
  if (wpc <= 0) wpc = 4;
  const long long target = (long long)di->n_cu * wpc;
  int n_items, n_waves, per = 0, chunks = 0;
  if (dim == 1) {
    n_items = (int)((cells + kStripWidth - 1) / kStripWidth);
    n_waves = (int)std::min<long long>(n_items, target);
  } else {
    const int ns = (nx + kStripWidth - 1) / kStripWidth;
    per = (int)std::max<long long>(4, ((long long)ns * ny + target - 1) / target);
    chunks = (ny + per - 1) / per;
    n_items = ns * chunks;
    n_waves = n_items;
  }
  const size_t off_items = up(kOffPtr + (size_t)(n_waves + 1) * sizeof(int));
  if (off_items + (size_t)n_items * sizeof(WorkItem) > kHeaderBytes) return HWENOU_ESCRATCH;

  unsigned char* base = di->ptr;
  unsigned char* data = base + kHeaderBytes;
  void* m_base = data;
  double* s1u = reinterpret_cast<double*>(data + mb);
  void* s1m = data + mb + ub;
  double* s2u = reinterpret_cast<double*>(data + mb + ub + mb);
  void* s2m = data + mb + 2 * ub + mb;
  int* status = status_dev ? status_dev : reinterpret_cast<int*>(base + kOffStatus);

  hipStream_t st = static_cast<hipStream_t>(stream);
  const int setup_threads = std::max(n_items, n_waves + 1);
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3((setup_threads + 255) / 256), dim3(256), 0, st,
                     base, inst_dev(d, *inst), dim, n_items, n_waves, per, chunks, off_items,
                     status_dev ? 0 : 1);
  if ((e = hipGetLastError()) != hipSuccess) return HWENOU_EHIP;

  const SchemeParams P = scheme_params(*d);
  auto run = [&](auto* tag) -> hipError_t {
    using TM = std::remove_pointer_t<decltype(tag)>;
    StageArgs<TM> A;
    A.P = P;
    A.inst = reinterpret_cast<const InstDev*>(base + kOffInst);
    A.dt = dt_dev;
    A.alpha = alpha_dev;
    A.done = nullptr;
    A.u_base = ubar;
    A.m_base = static_cast<TM*>(m_base);
    A.alpha_next = nullptr;
    A.alpha_slots = 1;
    A.status = status;
    A.plane = cells;
    A.work = reinterpret_cast<const WorkItem*>(base + off_items);
    A.work_ptr = reinterpret_cast<const int*>(base + kOffPtr);
    A.n_waves = n_waves;
    const double* uin[3] = {ubar, s1u, s2u};
    TM* min_[3] = {static_cast<TM*>(mom), static_cast<TM*>(s1m), static_cast<TM*>(s2m)};
    double* uout[3] = {s1u, s2u, ubar};
    TM* mout[3] = {static_cast<TM*>(s1m), static_cast<TM*>(s2m), static_cast<TM*>(mom)};
    for (int s = 0; s < 3; ++s) {
      A.stage = s;
      A.u_in = uin[s];
      A.m_in = min_[s];
      A.u_out = uout[s];
      A.m_out = mout[s];
      const hipError_t le =
          dim == 1 ? launch_stage_1d(d->eq, chr, mixed, &A, (n_waves + 3) / 4, 256, st)
                   : launch_stage_2d(d->eq, chr, mixed, si, &A, n_waves, 64, st);
      if (le != hipSuccess) return le;
    }
    return hipSuccess;
  };
  e = mixed ? run(static_cast<float*>(nullptr)) : run(static_cast<double*>(nullptr));
  return e == hipSuccess ? HWENOU_OK : HWENOU_EHIP;
}
