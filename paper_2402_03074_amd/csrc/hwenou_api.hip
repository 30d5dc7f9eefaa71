// Host side of libhwenou.so: handle management, work lists of the
// persistent stage launches, the stage entry point and the graph-replayed
// time loop.  See include/hwenou.h for the contract of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hwenou.h"
#include "hwenou_internal.hpp"

using namespace hwenou;

namespace {

thread_local char g_hip_error[256] = "";

int hip_fail(hipError_t e, const char* what) {
  std::snprintf(g_hip_error, sizeof g_hip_error, "HIP error in %s: %s", what,
                hipGetErrorString(e));
  return HWENOU_EHIP;
}

#define HIPCHK(call)                               \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

}  // namespace

struct hwenou_handle {
  hwenou_desc desc;
  int n_inst = 0;
  int dim = 1, nc = 1;
  bool mixed = false;
  long long plane = 0;
  size_t mom_elem = 8;
  hipStream_t stream = nullptr;      // caller's stream
  hipStream_t own = nullptr;         // capture stream of hwenou_advance
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hwenou_inst> inst;
  InstDev* d_inst = nullptr;
  // per-instance device state
  double *d_alpha = nullptr, *d_alpha_next = nullptr, *d_dt = nullptr, *d_t = nullptr;
  int *d_steps = nullptr, *d_done = nullptr, *d_status = nullptr, *d_all_done = nullptr;
  int* h_flags = nullptr;            // pinned [2]: all-done flags of the last two chunks
  RunParams* d_run = nullptr;        // parameters of the current hwenou_advance call
  RunParams* h_run = nullptr;        // pinned staging copy
  hipEvent_t ev_poll[2] = {nullptr, nullptr};
  // the step graphs of hwenou_advance (one step, and kMultiSteps steps in a
  // row), kept while the state pointers and the work lists stay the same
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  const void *g_ubar = nullptr, *g_mom = nullptr;
  // scratch of the time loop and the stage base
  void* m_base = nullptr;            // v^_n (w^_n) [dim][nc][plane]
  double *s1u = nullptr, *s2u = nullptr;
  void *s1m = nullptr, *s2m = nullptr;
  const double* u_base = nullptr;    // recorded by stage 0
  // work lists
  int waves_per_cu = 0, rows_per_item = 0;
  int n_cu = 256;
  int n_xcd = 8;  // chiplets, each with its own L2
  int alpha_slots = 1;  // wave-speed accumulators per instance
  WorkItem* d_work = nullptr;
  int* d_work_ptr = nullptr;
  int n_waves = 0;
  bool work_dirty = true;
};

namespace {

template <class T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e == hipErrorOutOfMemory) return HWENOU_ENOMEM;
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  return HWENOU_OK;
}

int dalloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e == hipErrorOutOfMemory) return HWENOU_ENOMEM;
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  return HWENOU_OK;
}

// Steps per replay of the multi-step graph: the gap between two graph
// launches (~5-10 us) then falls on every kMultiSteps-th step only, which
// matters for grids whose steps take tens of microseconds.
constexpr int kMultiSteps = 8;

void drop_graph(hwenou_handle* h) {
  for (int g = 0; g < 2; ++g) {
    if (h->exec[g]) (void)hipGraphExecDestroy(h->exec[g]);
    if (h->graph[g]) (void)hipGraphDestroy(h->graph[g]);
    h->exec[g] = nullptr;
    h->graph[g] = nullptr;
  }
  h->g_ubar = h->g_mom = nullptr;
}

void free_handle(hwenou_handle* h) {
  if (!h) return;
  drop_graph(h);
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(h->d_inst); f(h->d_alpha); f(h->d_alpha_next); f(h->d_dt); f(h->d_t);
  f(h->d_steps); f(h->d_done); f(h->d_status); f(h->d_all_done); f(h->d_run);
  f(h->m_base); f(h->s1u); f(h->s2u); f(h->s1m); f(h->s2m);
  f(h->d_work); f(h->d_work_ptr);
  if (h->h_flags) (void)hipHostFree(h->h_flags);
  if (h->h_run) (void)hipHostFree(h->h_run);
  for (hipEvent_t e : h->ev_poll)
    if (e) (void)hipEventDestroy(e);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  if (h->own) (void)hipStreamDestroy(h->own);
  delete h;
}

// Order the waves' runs for the chiplets.  The hardware hands the blocks of a
// launch to the XCDs in turn (block b to XCD b mod n_xcd), and every XCD has
// an L2 of its own.  The 2D work lists put runs that read the same cache
// lines next to each other (one grid: the strips of one band; many
// instances: consecutive rows of a strip, then the neighbouring strip), and
// here each XCD receives one contiguous range of the list.  For one grid the
// waves of neighbouring strips in a band then start together, march in step
// and share the columns at their common edge (the two-column halos and the
// cache lines a row segment straddles) through one L2, which fetches them
// from HBM once instead of once per XCD.
void xcd_order(std::vector<WorkItem>& items, std::vector<int>& ptr, int n_xcd) {
  const int nw = (int)ptr.size() - 1;
  if (n_xcd <= 1 || nw <= n_xcd) return;
  std::vector<int> run_of_block(nw);
  int r = 0;
  for (int x = 0; x < n_xcd; ++x)
    for (int b = x; b < nw; b += n_xcd) run_of_block[b] = r++;
  std::vector<WorkItem> it2;
  std::vector<int> p2;
  it2.reserve(items.size());
  p2.reserve(ptr.size());
  p2.push_back(0);
  for (int b = 0; b < nw; ++b) {
    const int q = run_of_block[b];
    for (int i = ptr[q]; i < ptr[q + 1]; ++i) it2.push_back(items[i]);
    p2.push_back((int)it2.size());
  }
  items.swap(it2);
  ptr.swap(p2);
}

// Build the per-wave work lists.
//  1D: tiles of kStripWidth cells; tiles are dealt out in contiguous runs.
//  2D, one grid (automatic shape): strips of kStripWidth columns, every strip
//      cut at the same rows into as many runs as fit the resident waves.
//  2D otherwise: the total strip-rows of all instances are split into equal
//      runs, one per wave, so every wave marches about the same number of
//      rows (a run that crosses the end of a strip continues at the bottom of
//      the next one).
// Also sets the number of wave-speed accumulators per instance.
int build_work(hwenou_handle* h) {
  drop_graph(h);  // the captured step graph holds the old work lists
  std::vector<WorkItem> items;
  std::vector<int> ptr;
  // default: as many waves per compute unit as can be resident at once
  int wpc = h->waves_per_cu;
  if (wpc <= 0) {
    const int chr = h->desc.eq == HWENOU_EQ_EULER ? h->desc.char_decomp : 0;
    const bool si = h->desc.weights == HWENOU_W_SCALE_INVARIANT;
    if (h->dim == 1)
      wpc = 4 * occupancy_stage_1d(h->desc.eq, chr, h->mixed, 256);
    else
      wpc = occupancy_stage_2d(h->desc.eq, chr, h->mixed, si, 64);
    if (wpc <= 0) wpc = 4;
  }
  const long long target_waves = (long long)h->n_cu * wpc;
  if (h->dim == 1) {
    std::vector<WorkItem> tiles;
    for (int k = 0; k < h->n_inst; ++k)
      for (int s = 0; s < h->inst[k].nx; s += kStripWidth) tiles.push_back({k, s, 0, 0});
    const long long nt = (long long)tiles.size();
    const long long nw = std::max<long long>(1, std::min<long long>(nt, target_waves));
    ptr.push_back(0);
    for (long long w = 0; w < nw; ++w) {
      const long long b = nt * (w + 1) / nw;
      ptr.push_back((int)b);
    }
    items = tiles;
  } else if (h->n_inst == 1 && h->rows_per_item <= 0) {
    // One grid: every strip is cut at the same rows into `q` runs of near-
    // equal length, and the runs are listed band by band.  The waves of one
    // band start together at the same row and march in step, so neighbouring
    // strips read their shared columns at the same time.
    const int ny = h->inst[0].ny;
    const int ns = (h->inst[0].nx + kStripWidth - 1) / kStripWidth;
    long long q = std::max<long long>(1, target_waves / ns);
    q = std::min<long long>(q, std::max(1, ny / 4));  // at least 4 rows per run
    ptr.push_back(0);
    for (long long b = 0; b < q; ++b) {
      const int r0 = (int)(ny * b / q), r1 = (int)(ny * (b + 1) / q);
      for (int s = 0; s < ns; ++s) {
        items.push_back({0, s, r0, r1});
        ptr.push_back((int)items.size());
      }
    }
    xcd_order(items, ptr, h->n_xcd);
  } else {
    struct Strip {
      int inst, strip, rows;
    };
    std::vector<Strip> strips;
    long long total = 0;
    for (int k = 0; k < h->n_inst; ++k) {
      const int ns = (h->inst[k].nx + kStripWidth - 1) / kStripWidth;
      for (int s = 0; s < ns; ++s) {
        strips.push_back({k, s, h->inst[k].ny});
        total += h->inst[k].ny;
      }
    }
    long long per = h->rows_per_item > 0 ? h->rows_per_item
                                         : (total + target_waves - 1) / target_waves;
    per = std::max<long long>(per, 4);
    ptr.push_back(0);
    long long used = 0;  // rows assigned to the current wave
    for (const Strip& s : strips) {
      int r = 0;
      while (r < s.rows) {
        const int take = (int)std::min<long long>(s.rows - r, per - used);
        items.push_back({s.inst, s.strip, r, r + take});
        r += take;
        used += take;
        if (used == per) {
          ptr.push_back((int)items.size());
          used = 0;
        }
      }
    }
    if (used > 0) ptr.push_back((int)items.size());
    xcd_order(items, ptr, h->n_xcd);
  }
  h->n_waves = (int)ptr.size() - 1;
  {
    // waves per instance, for the number of wave-speed accumulators
    std::vector<int> waves(h->n_inst, 0), last(h->n_inst, -1);
    for (int w = 0; w < h->n_waves; ++w)
      for (int i = ptr[w]; i < ptr[w + 1]; ++i) {
        const int k = items[i].inst;
        if (last[k] != w) {
          last[k] = w;
          ++waves[k];
        }
      }
    const int busiest = waves.empty() ? 0 : *std::max_element(waves.begin(), waves.end());
    int slots = 1;
    while (slots < kAlphaSlots && 64 * slots < busiest) slots *= 2;
    h->alpha_slots = slots;
  }
  if (h->d_work) (void)hipFree(h->d_work);
  if (h->d_work_ptr) (void)hipFree(h->d_work_ptr);
  h->d_work = nullptr;
  h->d_work_ptr = nullptr;
  int rc = dalloc(&h->d_work, items.size());
  if (rc) return rc;
  rc = dalloc(&h->d_work_ptr, ptr.size());
  if (rc) return rc;
  HIPCHK(hipMemcpy(h->d_work, items.data(), items.size() * sizeof(WorkItem),
                   hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_work_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
  h->work_dirty = false;
  return HWENOU_OK;
}

}  // namespace

SchemeParams hwenou::scheme_params(const hwenou_desc& d) {
  SchemeParams P;
  P.adv_x = d.adv[0];
  P.adv_y = d.adv[1];
  P.gas_gamma = d.gas_gamma;
  P.gamma_low = d.gamma_low;
  P.eps = d.eps;
  P.ave_mul = d.weights == HWENOU_W_ZQ ? 0.0 : 1.0;
  P.ave_add = d.weights == HWENOU_W_ZQ ? 1.0 : 0.0;
  P.nonlin = d.weights == HWENOU_W_LINEAR ? 0.0 : 1.0;
  return P;
}

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Wave-speed accumulators per instance (set with the work lists): one per
// 64 waves that work on the busiest instance, a power of two from 1 to
// kAlphaSlots.
int alpha_slots(const hwenou_handle* h) { return h->alpha_slots; }

int launch_stage(hwenou_handle* h, int s, const double* dt, const double* alpha, const int* done,
                 const double* u_in, const void* m_in, double* u_out, void* m_out,
                 double* alpha_next, hipStream_t st) {
  if (h->work_dirty) {
    int rc = build_work(h);
    if (rc) return rc;
  }
  const SchemeParams P = scheme_params(h->desc);
  const int chr = h->desc.eq == HWENOU_EQ_EULER ? h->desc.char_decomp : 0;
  const bool si = h->desc.weights == HWENOU_W_SCALE_INVARIANT;
  hipError_t e;
  auto fill = [&](auto& A, auto* mi, auto* mo, auto* mb) {
    A.P = P;
    A.inst = h->d_inst;
    A.dt = dt;
    A.alpha = alpha;
    A.done = done;
    A.u_in = u_in;
    A.m_in = mi;
    A.u_base = h->u_base;
    A.m_base = mb;
    A.u_out = u_out;
    A.m_out = mo;
    A.alpha_next = alpha_next;
    A.alpha_slots = alpha_slots(h);
    A.status = h->d_status;
    A.plane = h->plane;
    A.work = h->d_work;
    A.work_ptr = h->d_work_ptr;
    A.n_waves = h->n_waves;
    A.stage = s;
  };
  if (h->mixed) {
    StageArgs<float> A;
    fill(A, static_cast<const float*>(m_in), static_cast<float*>(m_out),
         static_cast<float*>(h->m_base));
    if (h->dim == 1)
      e = launch_stage_1d(h->desc.eq, chr, true, &A, (h->n_waves + 3) / 4, 256, st);
    else
      e = launch_stage_2d(h->desc.eq, chr, true, si, &A, h->n_waves, 64, st);
  } else {
    StageArgs<double> A;
    fill(A, static_cast<const double*>(m_in), static_cast<double*>(m_out),
         static_cast<double*>(h->m_base));
    if (h->dim == 1)
      e = launch_stage_1d(h->desc.eq, chr, false, &A, (h->n_waves + 3) / 4, 256, st);
    else
      e = launch_stage_2d(h->desc.eq, chr, false, si, &A, h->n_waves, 64, st);
  }
  if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  return HWENOU_OK;
}

AuxArgs aux_args(hwenou_handle* h, const double* u) {
  AuxArgs a;
  a.P = scheme_params(h->desc);
  a.eq = h->desc.eq;
  a.dim = h->dim;
  a.n_inst = h->n_inst;
  a.inst = h->d_inst;
  a.plane = h->plane;
  a.u = u;
  a.alpha = h->d_alpha;
  a.dt = h->d_dt;
  a.t = h->d_t;
  a.steps = h->d_steps;
  a.done = h->d_done;
  a.status = h->d_status;
  a.alpha_next = h->d_alpha_next;
  a.alpha_slots = alpha_slots(h);
  a.run = h->d_run;
  a.all_done = h->d_all_done;
  return a;
}

}  // namespace

namespace hwenou {

int check_desc(const hwenou_desc* d) {
  if (!d) return HWENOU_EINVAL;
  if (d->dim != 1 && d->dim != 2) return HWENOU_EINVAL;
  if (d->eq < HWENOU_EQ_ADVECTION || d->eq > HWENOU_EQ_EULER) return HWENOU_EINVAL;
  if (d->precision != HWENOU_FP64 && d->precision != HWENOU_MIXED) return HWENOU_EINVAL;
  if (d->weights < HWENOU_W_SCALE_INVARIANT || d->weights > HWENOU_W_LINEAR) return HWENOU_EINVAL;
  if (d->char_decomp < HWENOU_CHAR_COMPONENT || d->char_decomp > HWENOU_CHAR_INTERFACE)
    return HWENOU_EINVAL;
  if (d->char_decomp == HWENOU_CHAR_INTERFACE && d->eq == HWENOU_EQ_EULER && d->dim != 2)
    return HWENOU_EINVAL;
  if (!(d->gamma_low > 0.0) || d->gamma_low * (d->dim == 1 ? 2 : 4) >= 1.0) return HWENOU_EINVAL;
  if (!(d->eps >= 0.0)) return HWENOU_EINVAL;
  if (d->eq == HWENOU_EQ_EULER && !(d->gas_gamma > 1.0)) return HWENOU_EINVAL;
  return HWENOU_OK;
}

int check_inst(const hwenou_desc* d, const hwenou_inst& I) {
  const int ny = d->dim == 1 ? 1 : I.ny;
  if (I.nx < 3 || (d->dim == 2 && ny < 3)) return HWENOU_EINVAL;
  if (!(I.x1 > I.x0) || (d->dim == 2 && !(I.y1 > I.y0))) return HWENOU_EINVAL;
  for (int s = 0; s < 2 * d->dim; ++s)
    if (I.bc[s] != HWENOU_BC_PERIODIC && I.bc[s] != HWENOU_BC_TRANSMISSIVE &&
        !(I.bc[s] == HWENOU_BC_REFLECTIVE && d->eq == HWENOU_EQ_EULER))
      return HWENOU_EINVAL;
  if (I.offset < 0) return HWENOU_EINVAL;
  const long long n = (long long)I.nx * ny;
  if (n > (1LL << 29)) return HWENOU_EUNSUPPORTED;  // 32-bit byte offsets in the kernels
  return HWENOU_OK;
}

InstDev inst_dev(const hwenou_desc* d, const hwenou_inst& I) {
  InstDev r;
  r.nx = I.nx;
  r.ny = d->dim == 1 ? 1 : I.ny;
  for (int s = 0; s < 4; ++s) r.bc[s] = (s < 2 * d->dim) ? I.bc[s] : HWENOU_BC_PERIODIC;
  r.dx = (I.x1 - I.x0) / I.nx;
  r.dy = d->dim == 1 ? 1.0 : (I.y1 - I.y0) / I.ny;
  r.offset = I.offset;
  return r;
}

}  // namespace hwenou

extern "C" {

const char* hwenou_strerror(int code) {
  switch (code) {
    case HWENOU_OK: return "success";
    case HWENOU_EINVAL: return "invalid argument";
    case HWENOU_ENOMEM: return "out of device memory";
    case HWENOU_EHIP: return g_hip_error[0] ? g_hip_error : "HIP error";
    case HWENOU_ENONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
    case HWENOU_EUNSUPPORTED: return "unsupported configuration";
    case HWENOU_ESCRATCH:
      return "instance too large for the fixed scratch of hwenou_step_noalloc "
             "(HWENOU_NOALLOC_MAX_BYTES)";
    default: return "unknown error code";
  }
}


int hwenou_create(const hwenou_desc* d, int n_inst, const hwenou_inst* inst, void* stream,
                  hwenou_handle** out) {
  if (!out) return HWENOU_EINVAL;
  *out = nullptr;
  if (!d || !inst || n_inst < 1) return HWENOU_EINVAL;
  int rc0 = check_desc(d);
  if (rc0) return rc0;
  // instances: sizes, domains, boundary conditions, non-overlapping ranges
  std::vector<std::pair<long long, long long>> ranges;
  long long plane = 0;
  for (int k = 0; k < n_inst; ++k) {
    const hwenou_inst& I = inst[k];
    if ((rc0 = check_inst(d, I))) return rc0;
    const long long n = (long long)I.nx * (d->dim == 1 ? 1 : I.ny);
    ranges.push_back({I.offset, I.offset + n});
    plane = std::max(plane, (long long)(I.offset + n));
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t k = 1; k < ranges.size(); ++k)
    if (ranges[k].first < ranges[k - 1].second) return HWENOU_EINVAL;

  hwenou_handle* h = new hwenou_handle();
  h->desc = *d;
  if (d->dim == 1) {
    h->desc.adv[1] = 0.0;
  }
  h->n_inst = n_inst;
  h->dim = d->dim;
  h->nc = d->eq == HWENOU_EQ_EULER ? d->dim + 2 : 1;
  h->mixed = d->precision == HWENOU_MIXED;
  h->mom_elem = h->mixed ? 4 : 8;
  h->plane = plane;
  h->stream = static_cast<hipStream_t>(stream);
  h->inst.assign(inst, inst + n_inst);
  int dev = 0;
  hipDeviceProp_t prop;
  int rc = HWENOU_OK;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    free_handle(h);
    return hip_fail(e, "hipGetDeviceProperties");
  }
  h->n_cu = prop.multiProcessorCount;
  {
    int nx = 0;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && nx > 0)
      h->n_xcd = nx;
  }

  std::vector<InstDev> di(n_inst);
  for (int k = 0; k < n_inst; ++k) di[k] = inst_dev(d, inst[k]);
  const size_t mom_bytes = (size_t)h->dim * h->nc * plane * h->mom_elem;
  const size_t u_count = (size_t)h->nc * plane;
#define TRY(x)            \
  do {                    \
    rc = (x);             \
    if (rc) {             \
      free_handle(h);     \
      return rc;          \
    }                     \
  } while (0)
  TRY(dalloc(&h->d_inst, n_inst));
  TRY(dalloc(&h->d_alpha, 2 * n_inst));
  TRY(dalloc(&h->d_alpha_next, (size_t)kAlphaStride * kAlphaSlots * n_inst));
  TRY(dalloc(&h->d_dt, n_inst));
  TRY(dalloc(&h->d_t, n_inst));
  TRY(dalloc(&h->d_steps, n_inst));
  TRY(dalloc(&h->d_done, n_inst));
  TRY(dalloc(&h->d_status, n_inst));
  TRY(dalloc(&h->d_all_done, 1));
  TRY(dalloc(&h->d_run, 1));
  TRY(dalloc_bytes(&h->m_base, mom_bytes));
  TRY(dalloc(&h->s1u, u_count));
  TRY(dalloc(&h->s2u, u_count));
  TRY(dalloc_bytes(&h->s1m, mom_bytes));
  TRY(dalloc_bytes(&h->s2m, mom_bytes));
#undef TRY
  auto chk = [&](hipError_t e2, const char* what) {
    if (e2 != hipSuccess) {
      rc = hip_fail(e2, what);
      return false;
    }
    return true;
  };
  if (!chk(hipHostMalloc(reinterpret_cast<void**>(&h->h_flags), 2 * sizeof(int)), "hipHostMalloc") ||
      !chk(hipHostMalloc(reinterpret_cast<void**>(&h->h_run), sizeof(RunParams)), "hipHostMalloc") ||
      !chk(hipMemcpy(h->d_inst, di.data(), n_inst * sizeof(InstDev), hipMemcpyHostToDevice),
           "hipMemcpy") ||
      !chk(hipMemset(h->d_status, 0, n_inst * sizeof(int)), "hipMemset") ||
      !chk(hipEventCreateWithFlags(&h->ev_poll[0], hipEventDisableTiming), "hipEventCreate") ||
      !chk(hipEventCreateWithFlags(&h->ev_poll[1], hipEventDisableTiming), "hipEventCreate") ||
      !chk(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking), "hipStreamCreate") ||
      !chk(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming), "hipEventCreate") ||
      !chk(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming), "hipEventCreate")) {
    free_handle(h);
    return rc;
  }
  rc = build_work(h);
  if (rc) {
    free_handle(h);
    return rc;
  }
  *out = h;
  return HWENOU_OK;
}

int hwenou_destroy(hwenou_handle* h) {
  if (!h) return HWENOU_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  (void)hipStreamSynchronize(h->own);
  free_handle(h);
  return HWENOU_OK;
}

int hwenou_set_launch(hwenou_handle* h, int waves_per_cu, int rows_per_item) {
  if (!h || waves_per_cu < 1 || waves_per_cu > 32 || rows_per_item < 0) return HWENOU_EINVAL;
  h->waves_per_cu = waves_per_cu;
  h->rows_per_item = rows_per_item;
  h->work_dirty = true;
  return HWENOU_OK;
}

int hwenou_autotune(hwenou_handle* h, const double* ubar, const void* mom, int reps,
                    int* waves_per_cu, int* rows_per_item) {
  if (!h || !ubar || !mom || reps < 1 || !aligned(ubar, 8) || !aligned(mom, h->mom_elem))
    return HWENOU_EINVAL;
  const int chr = h->desc.eq == HWENOU_EQ_EULER ? h->desc.char_decomp : 0;
  const bool si = h->desc.weights == HWENOU_W_SCALE_INVARIANT;
  const int occ = h->dim == 1 ? 4 * occupancy_stage_1d(h->desc.eq, chr, h->mixed, 256)
                              : occupancy_stage_2d(h->desc.eq, chr, h->mixed, si, 64);
  const int base = occ > 0 ? occ : 4;
  std::vector<int> wpcs;
  for (int f : {1, 2, 4}) {
    const int w = std::min(32, base * f);
    if (std::find(wpcs.begin(), wpcs.end(), w) == wpcs.end()) wpcs.push_back(w);
  }
  if (base > 1) wpcs.push_back(std::max(1, base / 2));
  std::vector<int> rows = h->dim == 1 ? std::vector<int>{0} : std::vector<int>{0, 16, 32, 64};
  hipStream_t st = h->own;
  HIPCHK(hipEventRecord(h->ev_in, h->stream));
  HIPCHK(hipStreamWaitEvent(st, h->ev_in, 0));
  HIPCHK(hipMemsetAsync(h->d_dt, 0, h->n_inst * sizeof(double), st));
  AuxArgs a = aux_args(h, ubar);
  hipError_t e = launch_max_wavespeed(a, st);
  if (e != hipSuccess) return hip_fail(e, "max_wavespeed launch");
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  const int save_w = h->waves_per_cu, save_r = h->rows_per_item;
  float best = 1e30f;
  int bw = save_w, br = save_r;
  int rc = HWENOU_OK;
  for (int w : wpcs) {
    for (int r : rows) {
      h->waves_per_cu = w;
      h->rows_per_item = r;
      h->work_dirty = true;
      if ((rc = build_work(h))) break;
      std::vector<float> ts;
      for (int k = 0; k <= reps && !rc; ++k) {  // first launch warms up
        if (hipEventRecord(t0, st) != hipSuccess) rc = HWENOU_EHIP;
        if (!rc) rc = launch_stage(h, 0, h->d_dt, h->d_alpha, nullptr, ubar, mom, h->s1u, h->s1m,
                                   nullptr, st);
        if (!rc && hipEventRecord(t1, st) != hipSuccess) rc = HWENOU_EHIP;
        if (!rc && hipEventSynchronize(t1) != hipSuccess) rc = HWENOU_EHIP;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) rc = HWENOU_EHIP;
        if (!rc && k > 0) ts.push_back(ms);
      }
      if (rc) break;
      std::sort(ts.begin(), ts.end());
      const float med = ts[ts.size() / 2];
      if (med < best) {
        best = med;
        bw = w;
        br = r;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  h->waves_per_cu = rc ? save_w : bw;
  h->rows_per_item = rc ? save_r : br;
  h->work_dirty = true;
  h->u_base = nullptr;  // the timed stage-0 launches overwrote the stored v^n
  if (rc) return rc == HWENOU_EHIP ? hip_fail(hipGetLastError(), "autotune timing") : rc;
  HIPCHK(hipStreamSynchronize(st));
  if (waves_per_cu) *waves_per_cu = bw;
  if (rows_per_item) *rows_per_item = br;
  return HWENOU_OK;
}

int hwenou_max_wavespeed(hwenou_handle* h, const double* ubar, double* alpha_dev) {
  if (!h || !ubar || !alpha_dev || !aligned(ubar, 8) || !aligned(alpha_dev, 8))
    return HWENOU_EINVAL;
  AuxArgs a = aux_args(h, ubar);
  a.alpha = alpha_dev;
  hipError_t e = launch_max_wavespeed(a, h->stream);
  if (e != hipSuccess) return hip_fail(e, "max_wavespeed launch");
  return HWENOU_OK;
}

int hwenou_stage(hwenou_handle* h, int s, const double* dt_dev, const double* alpha_dev,
                 const double* ubar_in, const void* mom_in, double* ubar_out, void* mom_out) {
  if (!h || s < 0 || s > 2 || !dt_dev || !alpha_dev || !ubar_in || !mom_in || !ubar_out ||
      !mom_out)
    return HWENOU_EINVAL;
  if (!aligned(ubar_in, 8) || !aligned(ubar_out, 8) || !aligned(mom_in, h->mom_elem) ||
      !aligned(mom_out, h->mom_elem) || !aligned(dt_dev, 8) || !aligned(alpha_dev, 8))
    return HWENOU_EINVAL;
  if (ubar_in == ubar_out || mom_in == mom_out) return HWENOU_EINVAL;
  if (s == 0) h->u_base = ubar_in;
  if (s > 0 && h->u_base == nullptr) return HWENOU_EINVAL;
  return launch_stage(h, s, dt_dev, alpha_dev, nullptr, ubar_in, mom_in, ubar_out, mom_out,
                      nullptr, h->stream);
}

int hwenou_inst_status(hwenou_handle* h, int* flags) {
  if (!h) return HWENOU_EINVAL;
  std::vector<int> st(h->n_inst);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipStreamSynchronize(h->own));
  HIPCHK(hipMemcpy(st.data(), h->d_status, h->n_inst * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(h->d_status, 0, h->n_inst * sizeof(int)));
  int any = 0;
  for (int k = 0; k < h->n_inst; ++k) {
    if (flags) flags[k] = st[k] & 1;
    any |= st[k] & 1;
  }
  return any ? HWENOU_ENONPHYSICAL : HWENOU_OK;
}

int hwenou_status(hwenou_handle* h) { return hwenou_inst_status(h, nullptr); }

int hwenou_advance(hwenou_handle* h, double* ubar, void* mom, double cfl, double t_final,
                   int max_steps, double* t_out, int* steps_out) {
  if (!h || !ubar || !mom || !(cfl > 0.0) || !(t_final >= 0.0) || max_steps < 0)
    return HWENOU_EINVAL;
  if (!aligned(ubar, 8) || !aligned(mom, h->mom_elem)) return HWENOU_EINVAL;
  if (h->work_dirty) {
    int rc = build_work(h);
    if (rc) return rc;
  }
  hipStream_t st = h->own;
  // order after the caller's prior work
  HIPCHK(hipEventRecord(h->ev_in, h->stream));
  HIPCHK(hipStreamWaitEvent(st, h->ev_in, 0));
  // the previous call synchronised its stream, so the staging copy is free
  h->h_run->cfl = cfl;
  h->h_run->t_final = t_final;
  h->h_run->max_steps = max_steps;
  HIPCHK(hipMemcpyAsync(h->d_run, h->h_run, sizeof(RunParams), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(h->d_t, 0, h->n_inst * sizeof(double), st));
  HIPCHK(hipMemsetAsync(h->d_steps, 0, h->n_inst * sizeof(int), st));
  HIPCHK(hipMemsetAsync(h->d_done, 0, h->n_inst * sizeof(int), st));
  HIPCHK(hipMemsetAsync(h->d_status, 0, h->n_inst * sizeof(int), st));
  AuxArgs a = aux_args(h, ubar);
  hipError_t e = launch_max_wavespeed(a, st);
  if (e != hipSuccess) return hip_fail(e, "max_wavespeed launch");
  // the first step's dt; later ones are set by the finish kernel of the step before
  e = launch_dt(a, st);
  if (e != hipSuccess) return hip_fail(e, "dt launch");

  // whole steps (three stages and the finish kernel) as graphs, captured
  // once and replayed by every later call on the same state arrays
  if (h->exec[0] == nullptr || h->g_ubar != ubar || h->g_mom != mom) {
    drop_graph(h);
    for (int g = 0; g < 2; ++g) {
      const int nsteps = g == 0 ? 1 : kMultiSteps;
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      int rc = HWENOU_OK;
      for (int q = 0; q < nsteps && rc == HWENOU_OK; ++q) {
        rc = launch_stage(h, 0, h->d_dt, h->d_alpha, h->d_done, ubar, mom, h->s1u, h->s1m,
                          nullptr, st);
        if (rc) break;
        h->u_base = ubar;
        rc = launch_stage(h, 1, h->d_dt, h->d_alpha, h->d_done, h->s1u, h->s1m, h->s2u, h->s2m,
                          nullptr, st);
        if (rc) break;
        rc = launch_stage(h, 2, h->d_dt, h->d_alpha, h->d_done, h->s2u, h->s2m, ubar, mom,
                          h->d_alpha_next, st);
        if (rc) break;
        if ((e = launch_finish(a, st)) != hipSuccess) rc = hip_fail(e, "finish launch");
      }
      e = hipStreamEndCapture(st, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        drop_graph(h);
        return rc;
      }
      if (e != hipSuccess) {
        drop_graph(h);
        return hip_fail(e, "hipStreamEndCapture");
      }
      e = hipGraphInstantiate(&h->exec[g], graph, nullptr, nullptr, 0);
      h->graph[g] = graph;
      if (e != hipSuccess) {
        h->exec[g] = nullptr;
        drop_graph(h);
        return hip_fail(e, "hipGraphInstantiate");
      }
    }
    h->g_ubar = ubar;
    h->g_mom = mom;
  }
  // Replays in chunks of growing length (multi-step graphs, then single
  // steps for the rest of a chunk).  After each chunk the all-done flag is
  // copied to a pinned slot; the host waits only for the flag of the chunk
  // before, so the device never idles between chunks.  Steps replayed after
  // every instance is done are no-ops.
  int launched = 0, chunk = 2 * kMultiSteps, slot = 0, prev = -1;
  while (launched < max_steps && e == hipSuccess) {
    const int k = std::min(chunk, max_steps - launched);
    for (int r = 0; r + kMultiSteps <= k && e == hipSuccess; r += kMultiSteps)
      e = hipGraphLaunch(h->exec[1], st);
    for (int r = 0; r < k % kMultiSteps && e == hipSuccess; ++r) e = hipGraphLaunch(h->exec[0], st);
    if (e != hipSuccess) break;
    launched += k;
    e = hipMemcpyAsync(&h->h_flags[slot], h->d_all_done, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(h->ev_poll[slot], st);
    if (e != hipSuccess) break;
    if (prev >= 0) {
      e = hipEventSynchronize(h->ev_poll[prev]);
      if (e != hipSuccess || h->h_flags[prev]) break;
    }
    prev = slot;
    slot ^= 1;
    chunk = std::min(2 * chunk, 512);
  }
  h->u_base = nullptr;  // the steps' stage-0 launches overwrote the stored v^n
  if (e != hipSuccess) return hip_fail(e, "graph replay");
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> t(h->n_inst);
  std::vector<int> steps(h->n_inst), status(h->n_inst);
  HIPCHK(hipMemcpy(t.data(), h->d_t, h->n_inst * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(steps.data(), h->d_steps, h->n_inst * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(status.data(), h->d_status, h->n_inst * sizeof(int), hipMemcpyDeviceToHost));
  if (t_out) std::memcpy(t_out, t.data(), h->n_inst * sizeof(double));
  if (steps_out) std::memcpy(steps_out, steps.data(), h->n_inst * sizeof(int));
  // later work on the caller's stream sees the result
  HIPCHK(hipEventRecord(h->ev_out, st));
  HIPCHK(hipStreamWaitEvent(h->stream, h->ev_out, 0));
  for (int k = 0; k < h->n_inst; ++k)
    if (status[k] & 1) return HWENOU_ENONPHYSICAL;
  return HWENOU_OK;
}

}  // extern "C"
