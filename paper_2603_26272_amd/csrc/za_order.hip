// Sweeps of the fourth-, eighth- and tenth-order central-upwind schemes
// (r = 2, 4, 5; Appendix A) in FP64 with the general weight kernels (Z, Ai,
// p and linear weights decided at run time).  Same kernels and launch shapes
// as WENO-ZA6 with the stencil half-width as a template parameter.
#include "za_internal.hpp"

using namespace za;

namespace {

template <int SYS, int M, int R>
void x_sys(za_ctx* c, int mode, const SweepArgs& a) {
  const CfgArg<double> cfg = make_cfg<double>(c->prob);
  const int nseg = (a.g.nx + XS_CELLS - 1) / XS_CELLS;
  const long long waves = (long long)a.g.ny * nseg;
  const dim3 grid((unsigned)((waves + 3) / 4)), blk(256);
  switch (mode) {
    case MODE_FLUX: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, double, MODE_FLUX, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
    case MODE_RHS: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, double, MODE_RHS, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
    case MODE_LX: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, double, MODE_LX, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
    default: hipLaunchKernelGGL((k_sweep_x_any<SYS, M, double, MODE_STAGE, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
  }
}

template <int SYS, int M, int R>
void y_sys(za_ctx* c, int mode, const SweepArgs& a) {
  const CfgArg<double> cfg = make_cfg<double>(c->prob);
  const dim3 grid((unsigned)((a.g.nx + 63) / 64), (unsigned)((a.g.ny + a.ytile - 1) / a.ytile)), blk(256);
  switch (mode) {
    case MODE_FLUX: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, double, MODE_FLUX, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
    case MODE_RHS: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, double, MODE_RHS, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
    default: hipLaunchKernelGGL((k_sweep_y_any<SYS, M, double, MODE_STAGE, WV_GENERAL, R>), grid, blk, 0, c->stream, a, cfg); break;
  }
}

template <int R>
void x_order(za_ctx* c, int mode, const SweepArgs& a) {
  switch (c->prob.system) {
    case ZA_EULER:
      if (c->prob.dim == 1) x_sys<SYS_EULER, 3, R>(c, mode, a); else x_sys<SYS_EULER, 4, R>(c, mode, a);
      break;
    case ZA_ADVECTION: x_sys<SYS_ADV, 1, R>(c, mode, a); break;
    case ZA_BURGERS: x_sys<SYS_BURGERS, 1, R>(c, mode, a); break;
    default: x_sys<SYS_BUCKLEY, 1, R>(c, mode, a); break;
  }
}

template <int R>
void y_order(za_ctx* c, int mode, const SweepArgs& a) {
  switch (c->prob.system) {
    case ZA_EULER: y_sys<SYS_EULER, 4, R>(c, mode, a); break;
    case ZA_ADVECTION: y_sys<SYS_ADV, 1, R>(c, mode, a); break;
    case ZA_BURGERS: y_sys<SYS_BURGERS, 1, R>(c, mode, a); break;
    default: y_sys<SYS_BUCKLEY, 1, R>(c, mode, a); break;
  }
}

}  // namespace

void launch_x_order(za_ctx* c, int mode, const SweepArgs& a) {
  switch (order_of(c->prob)) {
    case 2: x_order<2>(c, mode, a); break;
    case 4: x_order<4>(c, mode, a); break;
    default: x_order<5>(c, mode, a); break;
  }
}

void launch_y_order(za_ctx* c, int mode, const SweepArgs& a) {
  switch (order_of(c->prob)) {
    case 2: y_order<2>(c, mode, a); break;
    case 4: y_order<4>(c, mode, a); break;
    default: y_order<5>(c, mode, a); break;
  }
}
