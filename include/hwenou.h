/*
 * hwenou.h -- C-ABI of the MI355X HWENO-U library (libhwenou.so).
 *
 * The library advances the zeroth- and first-order moments of hyperbolic
 * conservation laws with the fifth-order moment-based Hermite WENO scheme
 * with unified stencils (HWENO-U) of Fan, Qiu & Zhao, arXiv 2402.03074:
 *   - problem statement: Section 2.1 (1D: u_t + f(u)_x = 0 on a uniform grid
 *     of [a, b], cell averages u_i and first-order moments v_i) and
 *     Section 2.2 (2D: u_t + f(u)_x + g(u)_y = 0 on [a, b] x [c, d], moments
 *     u_ij, v_ij, w_ij);
 *   - spatial operator: Steps 1-3 of Sections 2.1 / 2.2 (reconstruction,
 *     smoothness indicators, scale-invariant nonlinear weights, moment
 *     modification) and the semi-discrete schemes Eq. (2.3) / (2.16) with
 *     Lax-Friedrichs fluxes;
 *   - time discretisation: the modified SSP-RK3 of Eq. (2.13) (Step 4), which
 *     uses the modified moments v^ (w^) in the Runge-Kutta bases;
 *   - Euler equations: local characteristic decomposition (Remark 2.2).
 *
 * Memory model.  All state arrays are device memory owned by the caller.
 * Several independent instances may share one handle; instance k occupies
 * cells [offset_k, offset_k + nx_k * ny_k) of every component plane, with x
 * the fastest index.  With P = the plane length (max over k of
 * offset_k + nx_k * ny_k):
 *   ubar : double [ncomp][P]                  cell averages
 *   mom  : T      [dim][ncomp][P]              first-order moments, d = 0 the
 *                                              x-moment v, d = 1 the y-moment w
 * T is double for HWENOU_FP64 and float for HWENOU_MIXED.  ncomp is 1 for
 * scalar laws, 3 (1D) or 4 (2D) for Euler (rho, rho u[, rho v], E).
 * Device arrays alpha [n_inst][2] (wave speeds in x and y) and dt [n_inst]
 * are doubles.  Pointers must be aligned to their element size.
 *
 * Every call is asynchronous on the handle's stream unless stated.  A handle
 * is not thread-safe.  Return values are HWENOU_OK or an error code below;
 * hwenou_strerror() describes a code (for HWENOU_EHIP, the last HIP error
 * text of the calling thread).
 */
#ifndef HWENOU_H
#define HWENOU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HWENOU_OK = 0,
  HWENOU_EINVAL = 1,        /* bad argument: enum, size, pointer alignment, order of calls */
  HWENOU_ENOMEM = 2,        /* device allocation failed */
  HWENOU_EHIP = 3,          /* a HIP call failed */
  HWENOU_ENONPHYSICAL = 4,  /* rho <= 0, p <= 0 or non-finite value after a stage */
  HWENOU_EUNSUPPORTED = 5,
  HWENOU_ESCRATCH = 6       /* hwenou_step_noalloc: instance beyond its fixed scratch */
};

enum { HWENOU_EQ_ADVECTION = 0, HWENOU_EQ_BURGERS = 1, HWENOU_EQ_EULER = 2 };
enum { HWENOU_FP64 = 0, HWENOU_MIXED = 1 };
/* nonlinear weights: scale-invariant (Eq. (2.11)/(2.22)), the scale-dependent
 * original (u_ave = 1, Remark 2.1 of Section 2.1), or linear (w = gamma). */
enum { HWENOU_W_SCALE_INVARIANT = 0, HWENOU_W_ZQ = 1, HWENOU_W_LINEAR = 2 };
/* Euler reconstruction variables (the local characteristic decomposition of
 * Remark 2.2, which leaves the state of the eigenvectors open): conserved
 * variables (component-wise); local characteristic variables at the cell's
 * own average in direction-split sweeps (x-edges, f and v^ from the
 * x-projection, y-edges, g and w^ from the y-projection; the default); one
 * reconstruction in x-characteristic variables for every output (2D; the
 * same as SPLIT in 1D); or the split sweeps with the edge values at each
 * interface in the characteristic variables of the Roe average of the two
 * cells that share it, the interior values and v^, w^ at the cell's own
 * average (2D Euler only; three reconstructions per cell and direction). */
enum {
  HWENOU_CHAR_COMPONENT = 0,
  HWENOU_CHAR_SPLIT = 1,
  HWENOU_CHAR_SINGLE = 2,
  HWENOU_CHAR_INTERFACE = 3
};
/* boundary conditions per side: periodic; transmissive (outflow: ghost cells
 * copy the boundary cell); reflective (Euler only: a solid wall, ghost cells
 * are mirror images with the wall-normal momentum negated and the moments
 * along the wall normal negated once more), the walls of the blast-wave and
 * Sedov problems of Section 3.2. */
enum { HWENOU_BC_PERIODIC = 0, HWENOU_BC_TRANSMISSIVE = 1, HWENOU_BC_REFLECTIVE = 2 };

/* Scheme description. */
typedef struct hwenou_desc {
  int dim;          /* 1 or 2 */
  int eq;           /* HWENOU_EQ_*; advection: f = adv[0] u, g = adv[1] u;
                       Burgers: f = g = u^2/2; Euler: ideal gas */
  int precision;    /* HWENOU_FP64 or HWENOU_MIXED (FP64 averages, smoothness
                       indicators and weights; FP32 moments, point values, fluxes) */
  int char_decomp;  /* Euler: HWENOU_CHAR_* */
  int weights;      /* HWENOU_W_* */
  double adv[2];    /* advection velocity */
  double gas_gamma; /* ratio of specific heats (Euler) */
  double gamma_low; /* linear weight of every linear polynomial (paper: 1/400) */
  double eps;       /* epsilon of the nonlinear weights (paper: 1e-10), >= 0.
                       The weights are evaluated with one reciprocal over the
                       product of the five (2D) or three (1D) denominators
                       beta_m u_ave + eps, scaled first by the power of two
                       that brings the quartic's denominator into [1, 2), so
                       the range follows the spread of the denominators, not
                       the magnitude of the state. */
} hwenou_desc;

/* One instance: a uniform grid of nx x ny cells on [x0, x1] x [y0, y1]
 * (ny = 1, y0/y1 ignored in 1D).  bc: x-lo, x-hi, y-lo, y-hi (HWENOU_BC_*).
 * Transmissive ghost cells copy the average and moments of the boundary cell. */
typedef struct hwenou_inst {
  int nx, ny;
  double x0, x1, y0, y1;
  int bc[4];
  int64_t offset;
} hwenou_inst;

typedef struct hwenou_handle hwenou_handle;

/* Create a handle for n_inst instances sharing one scheme description.
 * `stream` is a hipStream_t (NULL = the default stream); every later call is
 * ordered on it.  The handle owns its scratch: the stage buffers used by
 * hwenou_advance, the stored modified moments of stage 0, per-instance
 * alpha/dt/t/step arrays and the work lists.  Errors: EINVAL (dim, eq,
 * precision, weights or char_decomp out of range; n_inst < 1; nx or ny < 3;
 * overlapping instances; gas_gamma <= 1 for Euler; a reflective side for a
 * scalar law),
 * EUNSUPPORTED (an instance of more than 2^29 cells: the kernels address an
 * instance with 32-bit byte offsets), ENOMEM, EHIP.  On error *out is NULL. */
int hwenou_create(const hwenou_desc* desc, int n_inst, const hwenou_inst* inst, void* stream,
                  hwenou_handle** out);

/* Release the handle and its device memory (synchronises its stream). */
int hwenou_destroy(hwenou_handle* h);

/* Static description of an error code. */
const char* hwenou_strerror(int code);

/* alpha_dev[k][d] = max over the cells of instance k of |f_d'(u)| at the
 * cell averages (Euler: |u_d| + c), d < dim; the Lax-Friedrichs coefficient
 * of Section 2.1 and the CFL wave speed.  Asynchronous.  A non-physical
 * average is reported by the next hwenou_advance or hwenou_status call. */
int hwenou_max_wavespeed(hwenou_handle* h, const double* ubar, double* alpha_dev);

/* One fused stage s in {0, 1, 2} of the modified SSP-RK3 (Eq. (2.13)):
 *   s = 0: out = (u, v^) + dt F(in)                 with (u, v^) from `in`
 *   s = 1: out = 3/4 (u^n, v^n) + 1/4 ((u, v^) + dt F(in))
 *   s = 2: out = 1/3 (u^n, v^n) + 2/3 ((u, v^) + dt F(in))
 * where v^ (and w^) are the HWENO moment modifications of `in` and
 * (u^n, v^n) is the base of the step: stage 0 records ubar_in as u^n (it must
 * stay valid and unchanged until stage 2 has run, except that stage 2 may
 * write its output into it) and stores v^n in the handle.  dt_dev [n_inst]
 * and alpha_dev [n_inst][2] are device arrays.  `in` and `out` must not
 * alias.  hwenou_advance and hwenou_autotune run stage 0 themselves and clear
 * the record, so stage 1 or 2 then needs a new stage 0.  Asynchronous.
 * Errors: EINVAL (s out of range, stage 1/2 before stage 0, misaligned
 * pointer), EHIP. */
int hwenou_stage(hwenou_handle* h, int s, const double* dt_dev, const double* alpha_dev,
                 const double* ubar_in, const void* mom_in, double* ubar_out, void* mom_out);

/* Advance every instance in place until t_final or max_steps steps, with the
 * modified SSP-RK3 of Eq. (2.13) (Section 2.1, Step 4; Section 2.2, Step 4).
 * Each step takes alpha = max |f'(u)| (Lax-Friedrichs coefficient of
 * Eq. (2.4)) from the cell averages of U^n and the time step
 * dt = min(CFL dx / alpha, t_final - t) (1D) or CFL / (alpha_1/dx +
 * alpha_2/dy) clipped likewise (2D), or dt = t_final - t when every wave
 * speed of the instance is zero (all fluxes vanish).  The paper fixes the
 * CFL number (0.6 in Section 3) but not the formula; this is the usual one.
 * Whole steps (the three stages and a finish kernel that also sets the next
 * dt) are replayed from a HIP graph, with alpha and dt on the device; the
 * graph is captured on the first call and kept while the state pointers and
 * the launch shape stay the same.  The host reads a completion flag after
 * each chunk of steps without waiting for the chunk in flight, and
 * synchronises at the end.  An instance whose state leaves the physical
 * states (rho <= 0, p <= 0 or non-finite, flagged by any of its kernels)
 * stops after the step in which that happened: its t_out and steps_out
 * include that step, its arrays hold that step's result, and the other
 * instances go on.  t_out [n_inst] and steps_out [n_inst] are host arrays
 * (may be NULL).  Errors: EINVAL (cfl <= 0, t_final < 0, max_steps < 0,
 * misaligned pointer), ENONPHYSICAL (some instance stopped that way;
 * hwenou_inst_status tells which), EHIP. */
int hwenou_advance(hwenou_handle* h, double* ubar, void* mom, double cfl, double t_final,
                   int max_steps, double* t_out, int* steps_out);

/* Read and clear the per-instance status flags (synchronous): flags[k]
 * (host array [n_inst], may be NULL) is 1 if a kernel found a non-physical or
 * non-finite state of instance k since the flags were last cleared (by this
 * call, hwenou_status or the start of hwenou_advance), else 0.  Returns
 * HWENOU_OK, HWENOU_ENONPHYSICAL if any flag was set, or EHIP. */
int hwenou_inst_status(hwenou_handle* h, int* flags);

/* hwenou_inst_status without the per-instance flags. */
int hwenou_status(hwenou_handle* h);

/* Launch configuration of the stage kernels: waves per compute unit of the
 * persistent launch (1..32) and, in 2D, the rows a wave marches per work
 * item before the work list splits (0 = automatic: a handle of one grid cuts
 * every strip at the same rows and hands the runs to the chiplets in
 * contiguous ranges; a handle of many instances balances equal runs).  Used
 * by the autotuner; takes effect on the next call. */
int hwenou_set_launch(hwenou_handle* h, int waves_per_cu, int rows_per_item);

/* Autotuner of the persistent launch shape: times stage 0 on (ubar, mom)
 * (read only; output goes to handle scratch) for candidate waves per
 * compute unit (multiples of the resident count) and, in 2D, rows per work
 * item; keeps the fastest (median of `reps` timed launches) and returns it.
 * Synchronous.  Errors: EINVAL, EHIP. */
int hwenou_autotune(hwenou_handle* h, const double* ubar, const void* mom, int reps,
                    int* waves_per_cu, int* rows_per_item);

/* Size of the fixed device scratch of hwenou_step_noalloc: 64 MiB per device
 * (held from the first call on a device until the process ends). */
#define HWENOU_NOALLOC_MAX_BYTES 67108864

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One whole
 * step of the modified SSP-RK3 (Eq. (2.13)), the three stages of
 * hwenou_stage in order, of ONE instance (inst->offset must be 0), in place
 * on the caller's (ubar, mom), with the caller's device values dt_dev [1] and
 * alpha_dev [2]; no handle.  Every scratch buffer (the stored modified
 * moments, two stage buffers, the instance record and the work lists) lives
 * in one fixed device array of HWENOU_NOALLOC_MAX_BYTES per device, so the
 * call allocates nothing: about 256 bytes per cell for 2D Euler in FP64
 * (~250k cells, 500^2), 120 for 1D Euler.  Every call on a device shares that
 * array and rebuilds what it reads from it, so calls that overlap on one
 * device (other streams or threads) race: order them.  The first call on a
 * device looks up the array's address there (make it outside graph capture).
 * status_dev (device int, may be NULL) is OR-ed with 1 if a stage finds a
 * non-physical or non-finite state; it is not cleared.  Asynchronous on
 * `stream` (a hipStream_t, NULL = default).  Results equal those of
 * hwenou_stage with the same dt and alpha.  Errors: EINVAL (description,
 * instance, offset or a misaligned pointer), EUNSUPPORTED, ESCRATCH (the
 * instance does not fit the array), EHIP. */
int hwenou_step_noalloc(const hwenou_desc* desc, const hwenou_inst* inst, void* stream,
                        const double* dt_dev, const double* alpha_dev, double* ubar, void* mom,
                        int* status_dev);

#ifdef __cplusplus
}
#endif

#endif /* HWENOU_H */
