// libza: host side of the C ABI declared in include/za.h.
//
// One context = one problem shape on one device and stream.  It owns the
// RK3 stage states, the x-sweep partial RHS (2D), the wave-speed reduction
// partials and the device control block (LF speeds, dt, t) that lets whole
// RK3 steps run without host round trips.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "za.h"
#include "za_kernels.hpp"
#include "za_internal.hpp"

using namespace za;

namespace {

const char* kStatusStr[] = {"ok", "invalid argument", "out of device memory", "device error",
                            "non-finite or non-physical state", "unsupported", "busy"};

int ncomp_of(const za_problem& p) {
  if (p.system == ZA_EULER) return p.dim == 1 ? 3 : 4;
  return 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
za_status za_validate(const za_problem* p, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return ZA_ERR_ARG; };
  if (!p) return fail("problem is NULL");
  if (p->dim != 1 && p->dim != 2) return fail("dim must be 1 or 2");
  if (p->system < ZA_ADVECTION || p->system > ZA_BUCKLEY) return fail("unknown system");
  if (p->nx < 1 || p->ny < 1) return fail("nx and ny must be >= 1");
  if (p->dim == 1 && p->ny != 1) return fail("ny must be 1 in 1D");
  if ((long long)p->nx * p->ny > (1LL << 31)) return fail("grid too large");
  if (!(p->xhi > p->xlo) || (p->dim == 2 && !(p->yhi > p->ylo))) return fail("empty domain");
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return fail("unknown boundary condition");
  if (p->system == ZA_EULER && !(p->gamma > 1.0)) return fail("gamma must exceed 1");
  if (!(p->cfl > 0.0)) return fail("cfl must be positive");
  if (p->dt_rule < 0 || p->dt_rule > 1) return fail("unknown dt rule");
  if (p->precision < 0 || p->precision > 1) return fail("unknown precision");
  if (!(p->p >= 1.0)) return fail("p must be >= 1");
  if (!(p->eps > 0.0)) return fail("eps must be positive");
  if (p->affine_invariant && !(p->mu0 > 0.0)) return fail("mu0 must be positive");
  if (p->precision == ZA_FP32_RECON && (p->eps < 1e-37 || (p->affine_invariant && p->mu0 < 1e-18)))
    return fail("FP32 reconstruction needs eps >= 1e-37 and mu0 >= 1e-18 (normal FP32 range)");
  // 16 eps and (2 mu0)^2 must be normal FP64 numbers with a finite reciprocal
  if (p->precision == ZA_FP64 && (p->eps < 1e-300 || (p->affine_invariant && p->mu0 < 1e-150)))
    return fail("FP64 needs eps >= 1e-300 and mu0 >= 1e-150 (normal FP64 range)");
  if (p->order != 0 && (p->order < 2 || p->order > 5)) return fail("order r must be 2, 3, 4 or 5");
  if (p->pp_limiter != 0 && p->pp_limiter != 1) return fail("pp_limiter must be 0 or 1");
  if (p->alt_tau != 0 && p->alt_tau != 1) return fail("alt_tau must be 0 or 1");
  if (!(weight_L(*p) >= 0.0) || !(weight_L(*p) < 1e300)) return fail("weight_L must be finite and >= 0");
  if (!(weight_q(*p) >= 1.0) || !(weight_q(*p) < 1e300)) return fail("weight_q must be finite and >= 1");
  if (p->alt_tau && order_of(*p) != 3) {
    if (why) *why = "the alternative global indicator is defined here for r = 3 only";
    return ZA_ERR_UNSUPPORTED;
  }
  if (p->pp_limiter && p->system != ZA_EULER) return fail("the positivity limiter applies to the Euler equations");
  if (p->pp_limiter && (p->dt_rule != ZA_DT_CFL || p->cfl > 0.5))
    return fail("the positivity limiter needs the CFL time step with cfl <= 0.5");
  if (p->pp_limiter && order_of(*p) != 3) {
    if (why) *why = "the positivity limiter runs with r = 3 only";
    return ZA_ERR_UNSUPPORTED;
  }
  if (p->pp_limiter && p->precision != ZA_FP64) {
    if (why) *why = "the positivity limiter runs with FP64 reconstruction only";
    return ZA_ERR_UNSUPPORTED;
  }
  if (order_of(*p) != 3 && p->precision != ZA_FP64) {
    if (why) *why = "orders other than r = 3 run in FP64 only";
    return ZA_ERR_UNSUPPORTED;
  }
  return ZA_OK;
}

size_t za_state_count(const za_problem* p) {
  if (za_validate(p, nullptr) != ZA_OK) return 0;
  return (size_t)ncomp_of(*p) * p->nx * p->ny;
}

size_t za_workspace_bytes(const za_problem* p) {
  if (za_validate(p, nullptr) != ZA_OK) return 0;
  const size_t st = za_state_count(p) * sizeof(double);
  size_t b = 2 * st;                      // Q1, Q2
  if (p->dim == 2) b += st;               // L_x
  // reduction partials: at most one per stage-kernel block (bounded by the
  // grid), at least RED_BLOCKS_MAX
  const size_t blocks = p->dim == 2 ? (size_t)((p->nx + 63) / 64) * (size_t)((p->ny + 15) / 16)
                                    : (size_t)(((p->nx + XS_CELLS - 1) / XS_CELLS + 3) / 4);
  b += std::max<size_t>(RED_BLOCKS_MAX, blocks) * NPART * sizeof(double) + 4096 + sizeof(DevCtl);
  return b;
}

const char* za_status_str(za_status s) {
  int i = (int)s;
  if (i < 0 || i > 6) return "unknown status";
  return kStatusStr[i];
}

const char* za_ctx_last_error(const za_ctx* c) { return c ? c->err.c_str() : "no context"; }

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static za_status hip_fail(za_ctx* c, hipError_t e, const char* what) {
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ZA_ERR_NOMEM : ZA_ERR_DEVICE;
}

#define ZA_CHECK_LAUNCH(c, what)                              \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return hip_fail((c), e_, (what));   \
  } while (0)


static void timed_begin(za_ctx* c, int cls) {
  if (!c->timing) return;
  hipEvent_t e;
  hipEventCreate(&e);
  hipEventRecord(e, c->stream);
  c->ev_open[cls] = e;
}
static void timed_end(za_ctx* c, int cls) {
  if (!c->timing) return;
  hipEvent_t e;
  hipEventCreate(&e);
  hipEventRecord(e, c->stream);
  c->events[cls].push_back({c->ev_open[cls], e});
}

template <int SYS, int M, class T, int WV>
static void launch_x_t(za_ctx* c, int mode, const SweepArgs& a) {
  const CfgArg<T> cfg = make_cfg<T>(c->prob);
  const int nseg = (a.g.nx + XS_CELLS - 1) / XS_CELLS;
  const long long waves = (long long)a.g.ny * nseg;
  const dim3 grid((unsigned)((waves + 3) / 4)), blk(256);
  if constexpr (SYS == SYS_EULER && sizeof(T) == sizeof(double)) {
    if (c->ph.pp && (mode == MODE_LX || mode == MODE_STAGE)) {
      if (mode == MODE_LX)
        hipLaunchKernelGGL((k_sweep_x_pp<M, MODE_LX, WV>), grid, blk, 0, c->stream, a, cfg);
      else
        hipLaunchKernelGGL((k_sweep_x_pp<M, MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg);
      return;
    }
  }
  if constexpr (sizeof(T) == sizeof(double) && WV == WV_Z1) {
    if ((mode == MODE_LX || mode == MODE_STAGE) && a.xl_chunks > 0) {
      const long long w = xl_waves(a.g.nx, a.g.ny, a.xl_chunks);
      const dim3 gl((unsigned)((w + 3) / 4));
      if (mode == MODE_LX)
        hipLaunchKernelGGL((k_sweep_xl<SYS, M, WV, MODE_LX>), gl, blk, 0, c->stream, a, cfg);
      else
        hipLaunchKernelGGL((k_sweep_xl<SYS, M, WV, MODE_STAGE>), gl, blk, 0, c->stream, a, cfg);
      return;
    }
  }
  if constexpr (WV == WV_Z1) {
    switch (mode) {
      case MODE_FLUX: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, T, MODE_FLUX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_RHS: hipLaunchKernelGGL((k_sweep_x<SYS, M, T, MODE_RHS, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_LX: hipLaunchKernelGGL((k_sweep_x<SYS, M, T, MODE_LX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      default: hipLaunchKernelGGL((k_sweep_x<SYS, M, T, MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg); break;
    }
  } else {
    switch (mode) {
      case MODE_FLUX: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, T, MODE_FLUX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_RHS: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, T, MODE_RHS, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_LX: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, T, MODE_LX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      default: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, T, MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg); break;
    }
  }
}

template <int SYS, int M, class T, int WV>
static void launch_y_t(za_ctx* c, int mode, const SweepArgs& a) {
  const CfgArg<T> cfg = make_cfg<T>(c->prob);
  const dim3 grid((unsigned)((a.g.nx + 63) / 64), (unsigned)((a.g.ny + a.ytile - 1) / a.ytile)), blk(256);
  if constexpr (SYS == SYS_EULER && M == 4 && sizeof(T) == sizeof(double)) {
    if (c->ph.pp && mode == MODE_STAGE) {
      hipLaunchKernelGGL((k_sweep_y_pp<MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg);
      return;
    }
  }
  if constexpr (WV == WV_Z1) {
    switch (mode) {
      case MODE_FLUX: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, T, MODE_FLUX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_RHS: hipLaunchKernelGGL((k_sweep_y<SYS, M, T, MODE_RHS, WV>), grid, blk, 0, c->stream, a, cfg); break;
      default: hipLaunchKernelGGL((k_sweep_y<SYS, M, T, MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg); break;
    }
  } else {
    switch (mode) {
      case MODE_FLUX: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, T, MODE_FLUX, WV>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_RHS: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, T, MODE_RHS, WV>), grid, blk, 0, c->stream, a, cfg); break;
      default: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, T, MODE_STAGE, WV>), grid, blk, 0, c->stream, a, cfg); break;
    }
  }
}


// dispatch on (system, dim, precision, weight variant)
template <int SYS, int M>
static void launch_x_sys(za_ctx* c, int mode, const SweepArgs& a) {
  const bool gp = general_weights(c->prob);
  if (c->prob.precision == ZA_FP32_RECON) {
    if (gp) launch_x_t<SYS, M, float, WV_GENERAL>(c, mode, a); else launch_x_t<SYS, M, float, WV_Z1>(c, mode, a);
  } else {
    if (gp) launch_x_t<SYS, M, double, WV_GENERAL>(c, mode, a); else launch_x_t<SYS, M, double, WV_Z1>(c, mode, a);
  }
}
template <int SYS, int M>
static void launch_y_sys(za_ctx* c, int mode, const SweepArgs& a) {
  const bool gp = general_weights(c->prob);
  if (c->prob.precision == ZA_FP32_RECON) {
    if (gp) launch_y_t<SYS, M, float, WV_GENERAL>(c, mode, a); else launch_y_t<SYS, M, float, WV_Z1>(c, mode, a);
  } else {
    if (gp) launch_y_t<SYS, M, double, WV_GENERAL>(c, mode, a); else launch_y_t<SYS, M, double, WV_Z1>(c, mode, a);
  }
}

void launch_x(za_ctx* c, int mode, const SweepArgs& a) {
  timed_begin(c, 0);
  if (order_of(c->prob) != 3) {
    launch_x_order(c, mode, a);
    timed_end(c, 0);
    return;
  }
  switch (c->prob.system) {
    case ZA_EULER:
      if (c->prob.dim == 1) launch_x_sys<SYS_EULER, 3>(c, mode, a); else launch_x_sys<SYS_EULER, 4>(c, mode, a);
      break;
    case ZA_ADVECTION: launch_x_sys<SYS_ADV, 1>(c, mode, a); break;
    case ZA_BURGERS: launch_x_sys<SYS_BURGERS, 1>(c, mode, a); break;
    default: launch_x_sys<SYS_BUCKLEY, 1>(c, mode, a); break;
  }
  timed_end(c, 0);
}

void launch_y(za_ctx* c, int mode, const SweepArgs& a) {
  timed_begin(c, 1);
  if (order_of(c->prob) != 3) {
    launch_y_order(c, mode, a);
    timed_end(c, 1);
    return;
  }
  switch (c->prob.system) {
    case ZA_EULER: launch_y_sys<SYS_EULER, 4>(c, mode, a); break;
    case ZA_ADVECTION: launch_y_sys<SYS_ADV, 1>(c, mode, a); break;
    case ZA_BURGERS: launch_y_sys<SYS_BURGERS, 1>(c, mode, a); break;
    default: launch_y_sys<SYS_BUCKLEY, 1>(c, mode, a); break;
  }
  timed_end(c, 1);
}

static void launch_final(za_ctx* c, int kind, int nblk) {
  hipLaunchKernelGGL((k_wave_final<4>), dim3(1), dim3(256), 0, c->stream, c->part, nblk, c->ctl, c->geom, c->ph,
                     c->prob.dim, kind, (int)c->prob.system);
}

// Stand-alone wave-speed reduction of q followed by the final reduction.
void launch_wave(za_ctx* c, const double* q, int kind, int check_active) {
  timed_begin(c, 2);
  const size_t ncell = (size_t)c->prob.nx * c->prob.ny;
  const int nblk = c->red_blocks;
  switch (c->prob.system) {
    case ZA_EULER:
      if (c->prob.dim == 1)
        hipLaunchKernelGGL((k_wave_partial<SYS_EULER, 3>), dim3(nblk), dim3(256), 0, c->stream, q, ncell, c->ph, c->ctl, check_active, c->part);
      else
        hipLaunchKernelGGL((k_wave_partial<SYS_EULER, 4>), dim3(nblk), dim3(256), 0, c->stream, q, ncell, c->ph, c->ctl, check_active, c->part);
      break;
    case ZA_ADVECTION:
      hipLaunchKernelGGL((k_wave_partial<SYS_ADV, 1>), dim3(nblk), dim3(256), 0, c->stream, q, ncell, c->ph, c->ctl, check_active, c->part);
      break;
    case ZA_BURGERS:
      hipLaunchKernelGGL((k_wave_partial<SYS_BURGERS, 1>), dim3(nblk), dim3(256), 0, c->stream, q, ncell, c->ph, c->ctl, check_active, c->part);
      break;
    default:
      hipLaunchKernelGGL((k_wave_partial<SYS_BUCKLEY, 1>), dim3(nblk), dim3(256), 0, c->stream, q, ncell, c->ph, c->ctl, check_active, c->part);
      break;
  }
  launch_final(c, kind, nblk);
  timed_end(c, 2);
}

__global__ void k_ctl_init(DevCtl* ctl, DevCtl v) {
  if (threadIdx.x == 0) *ctl = v;
}
__global__ void k_ctl_arm(DevCtl* ctl, double dt_fixed, double t_final, long long max_steps) {
  // start a new stepping sequence from the current (t, steps)
  if (threadIdx.x != 0) return;
  ctl->dt_fixed = dt_fixed;
  ctl->t_final = t_final;
  ctl->max_steps = max_steps;
  ctl->active = ctl->bad ? 0 : 1;
}

SweepArgs base_args(za_ctx* c) {
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ctl = c->ctl;
  a.g = c->geom;
  a.ph = c->ph;
  a.ytile = c->ytile;
  a.part = nullptr;
  a.xl_chunks = c->xl_chunks;
  return a;
}

// Rows per y-sweep block: split each 64-column strip into as many tiles as
// there are resident block slots per strip, so that one round of blocks
// covers the grid (no tail round at partial occupancy).
template <class T>
static int pick_ytile(za_ctx* c) {
  const za_problem& p = c->prob;
  if (p.dim != 2) return 64;
  int blocks_per_cu = 0, cus = 0;
  const void* fn = p.system == ZA_EULER
                       ? reinterpret_cast<const void*>(&k_sweep_y<SYS_EULER, 4, T, MODE_STAGE, WV_Z1>)
                       : reinterpret_cast<const void*>(&k_sweep_y<SYS_ADV, 1, T, MODE_STAGE, WV_Z1>);
  if (order_of(p) != 3) {
    blocks_per_cu = order_y_blocks_per_cu(p);
  } else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, fn, 256, 0) != hipSuccess) {
    blocks_per_cu = 0;
  }
  if (blocks_per_cu < 1) blocks_per_cu = 2;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
    cus = 256;
  const long long strips = (p.nx + 63) / 64;
  const long long slots = (long long)blocks_per_cu * cus;
  long long tiles = std::max<long long>(1, slots / strips);
  // a tile of R rows computes R + 1 interface rows, YS_ROWS per step: take
  // the largest R with as many steps as the rows a tile needs
  const int need = (int)((p.ny + tiles - 1) / tiles);
  const int rows = YS_ROWS * ((need + YS_ROWS) / YS_ROWS) - 1;
  return std::max(rows, YS_TILE_MIN);
}

// Chunks per row segment of the looped x-sweep (stages in FP64, r = 3, Z
// weights with p = 1, no limiter; 0: the one-shot sweep).  A wavefront walks nc chunks of 64
// interfaces; the choice minimises rounds of resident wavefronts x chunks
// per wavefront (a record pass counted as 1/32 of a flux pass), i.e. the
// critical path when every SIMD slot is busy.
// ZA_XL_CHUNKS in the environment forces a value (0 disables the sweep).
static int pick_xl_chunks(za_ctx* c) {
  const za_problem& p = c->prob;
  if (p.precision != ZA_FP64 || order_of(p) != 3 || p.pp_limiter || general_weights(p)) return 0;
  if (const char* e = std::getenv("ZA_XL_CHUNKS")) {
    const int v = std::atoi(e);
    return v < 0 ? 0 : std::min(v, 256);
  }
  int blocks_per_cu = 0, cus = 0;
  const void* fn = p.system != ZA_EULER ? reinterpret_cast<const void*>(&k_sweep_xl<SYS_ADV, 1, WV_Z1, MODE_LX>)
                   : p.dim == 2         ? reinterpret_cast<const void*>(&k_sweep_xl<SYS_EULER, 4, WV_Z1, MODE_LX>)
                                        : reinterpret_cast<const void*>(&k_sweep_xl<SYS_EULER, 3, WV_Z1, MODE_STAGE>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, fn, 256, 0) != hipSuccess || blocks_per_cu < 1)
    blocks_per_cu = 3;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
    cus = 256;
  const long long slots = 4LL * blocks_per_cu * cus;
  int best = 1;
  long long best_cost = -1;
  for (int nc = 1; nc <= 64; ++nc) {
    const long long seg = 64LL * nc - 1;
    const long long waves = xl_waves(p.nx, p.ny, nc);
    const long long cost = ((waves + slots - 1) / slots) * (32LL * nc + nc + 1);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = nc; }
    if (seg >= p.nx) break;   // one segment per row from here on
  }
  return best;
}

// One RK3 step on the stream (no host synchronisation).  The kernel that
// writes a stage's new state also leaves the per-block wave-speed maxima of
// that state in c->part, so only the first step of an API call needs a
// stand-alone reduction pass.
// merge_end: the previous step deferred its end to this step's first final
// reduction; defer_end: leave this step's end to the next step.
static za_status enqueue_step(za_ctx* c, double* q, bool merge_end = false, bool defer_end = false) {
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  const double* in[3] = {q, c->q1, c->q2};
  double* out[3] = {c->q1, c->q2, q};
  for (int s = 0; s < 3; ++s) {
    const int kind = s == 0 ? FIN_STAGE0 : FIN_STAGEK;
    if (s == 0 && !c->speeds_valid) {
      if (merge_end) hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, c->stream, c->ctl);
      launch_wave(c, in[s], kind, 1);
    } else {
      launch_final(c, s == 0 && merge_end ? FIN_END_STAGE0 : kind, c->stage_blocks);
    }
    SweepArgs a = base_args(c);
    a.check_active = 1;
    a.q = in[s];
    a.qn = q;
    a.ca = ca[s];
    a.cb = cb[s];
    a.part = c->part;
    if (c->prob.dim == 1) {
      a.out = out[s];
      launch_x(c, MODE_STAGE, a);
    } else {
      a.out = c->lx;
      launch_x(c, MODE_LX, a);
      a.lx = c->lx;
      a.out = out[s];
      launch_y(c, MODE_STAGE, a);
    }
  }
  if (!defer_end) hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, c->stream, c->ctl);
  c->speeds_valid = true;
  ZA_CHECK_LAUNCH(c, "step launch");
  return ZA_OK;
}

// n RK3 steps.  After the first step of an API call (which may need the
// stand-alone wave-speed pass), runs of GRAPH_STEPS steps replay a hipGraph
// captured once per state pointer on a private capture stream; kernels read
// dt and the LF speeds from the device control block, so a graph is valid
// for any step.  Kernel timing (events) uses direct launches.
static constexpr int GRAPH_STEPS = 16;

static za_status enqueue_steps(za_ctx* c, double* q, int64_t n) {
  za_status st;
  int64_t done = 0;
  if (n > 0 && !c->speeds_valid) {
    if ((st = enqueue_step(c, q)) != ZA_OK) return st;
    done = 1;
  }
  if (!c->timing && c->graphs_ok && n - done >= GRAPH_STEPS) {
    if (!c->graph_exec || c->graph_q != q) {
      if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
      if (!c->capture_stream && hipStreamCreate(&c->capture_stream) != hipSuccess) c->graphs_ok = false;
      if (c->graphs_ok) {
        hipStream_t user = c->stream;
        c->stream = c->capture_stream;
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        // inside the graph each step's end runs with the next step's first
        // final reduction; the graph's last step ends on its own
        for (int i = 0; ok && i < GRAPH_STEPS; ++i)
          ok = enqueue_step(c, q, i > 0, i + 1 < GRAPH_STEPS) == ZA_OK;
        ok = (hipStreamEndCapture(c->stream, &g) == hipSuccess) && ok;
        c->stream = user;
        if (ok) ok = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
          c->graphs_ok = false;
          c->graph_exec = nullptr;
          (void)hipGetLastError();
        } else {
          c->graph_q = q;
        }
      }
    }
    while (c->graph_exec && n - done >= GRAPH_STEPS) {
      hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "graph launch");
      done += GRAPH_STEPS;
    }
  }
  for (bool pending = false; done < n; ++done) {
    const bool defer = done + 1 < n;
    if ((st = enqueue_step(c, q, pending, defer)) != ZA_OK) return st;
    pending = defer;
  }
  return ZA_OK;
}

static DevCtl fresh_ctl() {
  DevCtl v;
  std::memset(&v, 0, sizeof(v));
  v.t = 0.0;
  v.t_final = std::numeric_limits<double>::infinity();
  v.dt_min = std::numeric_limits<double>::infinity();
  v.dt_max = 0.0;
  v.bad_step = -1;
  v.active = 0;
  return v;
}

void launch_ctl_reset(za_ctx* c) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl, fresh_ctl());
}

// Everything a context derives from its problem without allocating: the
// geometry and physics constants, launch shapes and reduction sizes.
void init_shape(za_ctx* c, const za_problem* p, hipStream_t stream) {
  c->prob = *p;
  c->m = ncomp_of(*p);
  c->stream = stream;
  (void)hipGetDevice(&c->device);
  const size_t ncell = (size_t)p->nx * p->ny;
  c->geom.nx = p->nx;
  c->geom.ny = p->ny;
  c->geom.bc_x = p->bc_x;
  c->geom.bc_y = p->bc_y;
  c->geom.dx = (p->xhi - p->xlo) / p->nx;
  c->geom.dy = p->dim == 2 ? (p->yhi - p->ylo) / p->ny : 1.0;
  c->geom.inv_dx = 1.0 / c->geom.dx;
  c->geom.inv_dy = 1.0 / c->geom.dy;
  c->ph.gamma = p->gamma;
  c->ph.gm1 = p->gamma - 1.0;
  c->ph.adv[0] = p->adv_speed[0];
  c->ph.adv[1] = p->adv_speed[1];
  c->ph.cfl = p->cfl;
  c->ph.dt_rule = p->dt_rule;
  c->ph.lf_scalar = p->lf == ZA_LF_SCALAR ? 1 : 0;
  c->ph.pp = p->pp_limiter ? 1 : 0;
  c->red_blocks = (int)std::min<size_t>(RED_BLOCKS_MAX, std::max<size_t>(1, (ncell + 2047) / 2048));
  c->ytile = p->precision == ZA_FP32_RECON ? pick_ytile<float>(c) : pick_ytile<double>(c);
  c->xl_chunks = pick_xl_chunks(c);
  if (p->dim == 2) {
    c->stage_blocks = ((p->nx + 63) / 64) * ((p->ny + c->ytile - 1) / c->ytile);
  } else if (c->xl_chunks > 0) {   // one row of maxima per wavefront of the looped sweep
    c->stage_blocks = (int)xl_waves(p->nx, p->ny, c->xl_chunks);
  } else {
    const long long nseg = (p->nx + XS_CELLS - 1) / XS_CELLS;
    c->stage_blocks = (int)((nseg * p->ny + 3) / 4);
  }
  c->part_blocks = std::max(RED_BLOCKS_MAX, c->stage_blocks);
  // ZA_STEP_GRAPHS=0 runs the steps of za_solve as direct launches instead
  // of replaying captured step graphs (results are identical)
  if (const char* e = std::getenv("ZA_STEP_GRAPHS")) c->graphs_ok = std::atoi(e) != 0;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

za_status za_ctx_create(const za_problem* p, void* stream, za_ctx** out) {
  if (!out) return ZA_ERR_ARG;
  *out = nullptr;
  std::string why;
  za_status st = za_validate(p, &why);
  if (st != ZA_OK) return st;
  za_ctx* c = new za_ctx();
  init_shape(c, p, (hipStream_t)stream);
  const size_t st_bytes = (size_t)c->m * p->nx * p->ny * sizeof(double);
  hipError_t e;
  void* ptr = nullptr;
  if ((e = hipMalloc(&ptr, st_bytes)) != hipSuccess) { delete c; return ZA_ERR_NOMEM; }
  c->q1 = (double*)ptr;
  if ((e = hipMalloc(&ptr, st_bytes)) != hipSuccess) { za_ctx_destroy(c); return ZA_ERR_NOMEM; }
  c->q2 = (double*)ptr;
  if (p->dim == 2) {
    if ((e = hipMalloc(&ptr, st_bytes)) != hipSuccess) { za_ctx_destroy(c); return ZA_ERR_NOMEM; }
    c->lx = (double*)ptr;
  }
  if ((e = hipMalloc(&ptr, (size_t)c->part_blocks * NPART * sizeof(double) + 4096)) != hipSuccess) {
    za_ctx_destroy(c);
    return ZA_ERR_NOMEM;
  }
  c->part = (double*)ptr;
  if ((e = hipMalloc(&ptr, sizeof(DevCtl))) != hipSuccess) { za_ctx_destroy(c); return ZA_ERR_NOMEM; }
  c->ctl = (DevCtl*)ptr;
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl, fresh_ctl());
  if ((e = hipGetLastError()) != hipSuccess) { za_ctx_destroy(c); return ZA_ERR_DEVICE; }
  *out = c;
  return ZA_OK;
}

za_status za_ctx_destroy(za_ctx* c) {
  if (!c) return ZA_ERR_ARG;
  if (c->stream || true) hipStreamSynchronize(c->stream);
  for (int k = 0; k < 3; ++k) {
    for (auto& pr : c->events[k]) { hipEventDestroy(pr.first); hipEventDestroy(pr.second); }
  }
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->q1) hipFree(c->q1);
  if (c->q2) hipFree(c->q2);
  if (c->lx) hipFree(c->lx);
  if (c->part) hipFree(c->part);
  if (c->ctl) hipFree(c->ctl);
  delete c;
  return ZA_OK;
}

za_status za_ctx_set_stream(za_ctx* c, void* stream) {
  if (!c) return ZA_ERR_ARG;
  c->stream = (hipStream_t)stream;
  return ZA_OK;
}

za_status za_rhs(za_ctx* c, const double* q, double* rhs) {
  if (!c || !q || !rhs || q == rhs) return ZA_ERR_ARG;
  c->speeds_valid = false;
  launch_wave(c, q, FIN_RHS, 0);
  SweepArgs a = base_args(c);
  a.q = q;
  a.out = rhs;
  launch_x(c, MODE_RHS, a);
  if (c->prob.dim == 2) {
    a.lx = rhs;
    launch_y(c, MODE_RHS, a);
  }
  ZA_CHECK_LAUNCH(c, "rhs launch");
  return ZA_OK;
}

za_status za_rhs_fluxes(za_ctx* c, const double* q, double* fx, double* fy) {
  if (!c || !q || !fx) return ZA_ERR_ARG;
  c->speeds_valid = false;
  launch_wave(c, q, FIN_RHS, 0);
  SweepArgs a = base_args(c);
  a.q = q;
  a.out = fx;
  launch_x(c, MODE_FLUX, a);
  if (c->prob.dim == 2 && fy) {
    a.out = fy;
    launch_y(c, MODE_FLUX, a);
  }
  ZA_CHECK_LAUNCH(c, "flux launch");
  return ZA_OK;
}

static za_status read_ctl(za_ctx* c, DevCtl* h) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronise");
  e = hipMemcpy(h, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read control block");
  return ZA_OK;
}

za_status za_step(za_ctx* c, double* q, double dt, double* dt_used) {
  if (!c || !q) return ZA_ERR_ARG;
  c->speeds_valid = false;
  if (!(dt > 0.0) && !(dt <= 0.0)) return ZA_ERR_ARG;  // NaN
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl, fresh_ctl());
  hipLaunchKernelGGL(k_ctl_arm, dim3(1), dim3(64), 0, c->stream, c->ctl, dt > 0.0 ? dt : 0.0,
                     std::numeric_limits<double>::infinity(), 1LL);
  za_status st = enqueue_step(c, q);
  if (st != ZA_OK) return st;
  if (dt_used) {
    DevCtl h;
    if ((st = read_ctl(c, &h)) != ZA_OK) return st;
    *dt_used = h.dt;
    if (h.bad) return ZA_ERR_NONFINITE;
  }
  return ZA_OK;
}

za_status za_solve(za_ctx* c, double* q, double t_final, int64_t max_steps, za_solve_info* info) {
  if (!c || !q) return ZA_ERR_ARG;
  c->speeds_valid = false;
  if (!(t_final > 0.0) && max_steps <= 0) return ZA_ERR_ARG;
  if (t_final != t_final) return ZA_ERR_ARG;
  const auto& p = c->prob;
  DevCtl h;
  za_status st;
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl, fresh_ctl());
  const int chunk = c->chunk_steps > 0 ? c->chunk_steps : 32;
  if (t_final > 0.0 && p.dt_rule == ZA_DT_CFL_H2) {
    // fixed dt = cfl h^2: n equal steps, the last one lands on t_final
    const double h2 = p.dim == 2 ? std::min(c->geom.dx, c->geom.dy) : c->geom.dx;
    const double dt = p.cfl * h2 * h2;
    const int64_t n = (int64_t)std::ceil(t_final / dt * (1.0 - 1e-12));
    int64_t n_run = n;
    if (max_steps > 0 && max_steps < n) n_run = max_steps;
    const int64_t n_equal = std::min<int64_t>(n_run, n - 1);
    hipLaunchKernelGGL(k_ctl_arm, dim3(1), dim3(64), 0, c->stream, c->ctl, dt,
                       std::numeric_limits<double>::infinity(), (long long)n_equal);
    for (int64_t s = 0; s < n_equal;) {
      const int64_t k = std::min<int64_t>(n_equal - s, 64 * (int64_t)chunk);
      if ((st = enqueue_steps(c, q, k)) != ZA_OK) return st;
      s += k;
      if (s < n_equal) {
        if ((st = read_ctl(c, &h)) != ZA_OK) return st;
        if (h.bad) break;
      }
    }
    if (n_run == n) {
      const double last = t_final - (double)(n - 1) * dt;
      hipLaunchKernelGGL(k_ctl_arm, dim3(1), dim3(64), 0, c->stream, c->ctl, last,
                         std::numeric_limits<double>::infinity(), (long long)n);
      if ((st = enqueue_step(c, q)) != ZA_OK) return st;
    }
    if ((st = read_ctl(c, &h)) != ZA_OK) return st;
    if (n_run == n && !h.bad) h.t = t_final;
  } else {
    const double tf = t_final > 0.0 ? t_final : std::numeric_limits<double>::infinity();
    hipLaunchKernelGGL(k_ctl_arm, dim3(1), dim3(64), 0, c->stream, c->ctl, 0.0, tf,
                       (long long)(max_steps > 0 ? max_steps : 0));
    // A fixed step count is enqueued exactly; integrating to t_final
    // enqueues chunks and lets the device retire the steps beyond t_final.
    int64_t enqueued = 0;
    while (true) {
      int n = chunk;
      if (t_final <= 0.0) n = (int)std::min<int64_t>(chunk, max_steps - enqueued);
      if ((st = enqueue_steps(c, q, n)) != ZA_OK) return st;
      enqueued += n;
      if ((st = read_ctl(c, &h)) != ZA_OK) return st;
      if (!h.active || h.bad) break;
      if (t_final <= 0.0 && enqueued >= max_steps) break;
    }
  }
  if (info) {
    info->steps = h.steps;
    info->t = h.t;
    info->dt_min = h.dt_min;
    info->dt_max = h.dt_max;
    info->nonfinite_step = h.bad ? h.bad_step : -1;
  }
  return h.bad ? ZA_ERR_NONFINITE : ZA_OK;
}

za_status za_conserved_sums(za_ctx* c, const double* q, double* sums) {
  if (!c || !q || !sums) return ZA_ERR_ARG;
  c->speeds_valid = false;
  const size_t ncell = (size_t)c->prob.nx * c->prob.ny;
  const int nblk = (int)std::min<size_t>((size_t)c->part_blocks * NPART, std::max<size_t>(1, (ncell + 4095) / 4096));
  const size_t chunk = (ncell + nblk - 1) / nblk;
  std::vector<double> part(nblk);
  for (int comp = 0; comp < c->m; ++comp) {
    hipLaunchKernelGGL(k_sum_partial, dim3(nblk), dim3(256), 0, c->stream, q + comp * ncell, ncell, chunk, c->part);
    ZA_CHECK_LAUNCH(c, "sum launch");
    hipError_t e = hipMemcpyAsync(part.data(), c->part, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy sums");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "synchronise");
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    sums[comp] = s;
  }
  return ZA_OK;
}

za_status za_ctx_set_timing(za_ctx* c, int32_t enable) {
  if (!c) return ZA_ERR_ARG;
  c->timing = enable != 0;
  return ZA_OK;
}

za_status za_ctx_kernel_times(za_ctx* c, double* avg_ms, int64_t* counts) {
  if (!c || !avg_ms) return ZA_ERR_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronise");
  for (int k = 0; k < 3; ++k) {
    double tot = 0.0;
    for (auto& pr : c->events[k]) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, pr.first, pr.second);
      tot += ms;
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    const size_t n = c->events[k].size();
    avg_ms[k] = n ? tot / (double)n : 0.0;
    if (counts) counts[k] = (int64_t)n;
    c->events[k].clear();
  }
  return ZA_OK;
}

}  // extern "C"
