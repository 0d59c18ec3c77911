// Library-internal context layout (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "za.h"
#include "za_kernels.hpp"

struct za_ctx {
  za_problem prob;
  int m = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  za::Geom geom;
  za::Phys ph;
  double* q1 = nullptr;      // RK3 stage 1 state
  double* q2 = nullptr;      // RK3 stage 2 state
  double* lx = nullptr;      // 2D: x-sweep partial RHS
  double* part = nullptr;    // reduction partials
  za::DevCtl* ctl = nullptr; // device control block
  int red_blocks = 1;
  int ytile = 64;            // y-sweep rows per block
  int xl_chunks = 0;         // looped x-sweep chunks per row segment (0: one-shot sweep)
  int stage_blocks = 1;      // blocks of the kernel that writes a stage state
  int part_blocks = 1;       // capacity of `part` in blocks
  bool speeds_valid = false; // part holds the wave speeds of the current q
  bool graphs_ok = true;     // step graphs usable on this device
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;  // GRAPH_STEPS steps for state graph_q
  const double* graph_q = nullptr;
  int chunk_steps = 0;       // steps per host check in za_solve (0: default)
  bool timing = false;
  hipEvent_t ev_open[3] = {nullptr, nullptr, nullptr};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[3];
  std::string err;
};

za_status za_validate(const za_problem* p, std::string* why);

// r of the order-2r scheme (0 selects WENO-ZA6, r = 3)
inline int order_of(const za_problem& p) { return p.order == 0 ? 3 : p.order; }

// Z weights with p = 1 and mu = 1 take the fast kernels; Ai, p != 1, tau'
// and the linear-weight test mode take the general ones.
// L and q of eq:weights_unnormalized (both 0 select the paper's 1, 1)
inline double weight_L(const za_problem& p) { return p.weight_L == 0.0 && p.weight_q == 0.0 ? 1.0 : p.weight_L; }
inline double weight_q(const za_problem& p) { return p.weight_L == 0.0 && p.weight_q == 0.0 ? 1.0 : p.weight_q; }

// FP64 Z-weight kernels apply eps unscaled to the characteristic fields they
// carry scaled (Euler's acoustic fields, by 2c); that is exact to ~2e-13 of
// a stencil's scale only for eps up to the paper's 1e-40, so a larger eps
// takes the general kernels, which scale it.  They also form products of
// four indicators, which for a flat stencil are (16 eps)^4: below
// kEpsFastMin that product leaves the normal range (at eps ~ 1e-82 it is
// zero and the weights 0/0), so a smaller eps takes the general kernels too,
// which divide per indicator.
constexpr double kEpsFastMax = 1e-40;
constexpr double kEpsFastMin = 1e-70;

inline bool general_weights(const za_problem& p) {
  return p.p != 1.0 || p.affine_invariant || p.linear_weights || p.alt_tau || weight_L(p) != 1.0 ||
         weight_q(p) != 1.0 || (p.precision == ZA_FP64 && (p.eps > kEpsFastMax || p.eps < kEpsFastMin));
}

template <class T>
inline za::CfgArg<T> make_cfg(const za_problem& p) {
  za::CfgArg<T> c;
  // exact power-of-two rescalings of the reconstruction (see za6() and zar())
  c.w.eps16 = (T)(16.0 * p.eps);
  c.w.eps6 = (T)(6.0 * p.eps);
  c.w.eps6q = (T)(1.5 * p.eps);
  c.w.eps4 = (T)(4.0 * p.eps);
  c.w.eps1 = (T)p.eps;
  c.w.mu0x2 = (T)(2.0 * p.mu0);
  c.w.p = (T)p.p;
  c.w.ai = p.affine_invariant;
  c.w.linear = p.linear_weights;
  c.w.alt_tau = p.alt_tau;
  c.w.L = (T)weight_L(p);
  c.w.q = (T)weight_q(p);
  c.w.pq = (T)(p.p * weight_q(p));
  return c;
}

// Sweeps of the order-2r schemes with r != 3 (za_order.hip): FP64, general
// weights, every mode; `a` as for the r = 3 kernels.
void launch_x_order(za_ctx* c, int mode, const za::SweepArgs& a);
void launch_y_order(za_ctx* c, int mode, const za::SweepArgs& a);
int order_y_blocks_per_cu(const za_problem& p);

// Host-side building blocks of the right-hand side (za_lib.hip), shared with
// other entry points of the library.
void init_shape(za_ctx* c, const za_problem* p, hipStream_t stream);
za::SweepArgs base_args(za_ctx* c);
void launch_wave(za_ctx* c, const double* q, int kind, int check_active);
void launch_x(za_ctx* c, int mode, const za::SweepArgs& a);
void launch_y(za_ctx* c, int mode, const za::SweepArgs& a);
// reset the control block c->ctl on c->stream (a kernel, no memset)
void launch_ctl_reset(za_ctx* c);
