// Sweeps of the fourth-, eighth- and tenth-order central-upwind schemes
// (r = 2, 4, 5; Appendix A) in FP64: the WENO-ZA6 kernels and launch shapes
// with the stencil half-width as a template parameter; Z weights with an
// occupancy target, the other weight variants (and flux output) through the
// general kernels.
#include "za_internal.hpp"

using namespace za;

namespace {

// resident wavefronts per SIMD requested for the Z-weight kernels
template <int R> struct OrderWaves;
template <> struct OrderWaves<2> { enum { x = 5, y = 3 }; };
template <> struct OrderWaves<4> { enum { x = 3, y = 2 }; };
template <> struct OrderWaves<5> { enum { x = 2, y = 2 }; };

// Z weights with p = 1 take the occupancy-targeted kernels; Ai, p != 1 and
// linear weights the general ones.

template <int SYS, int M, int R>
void x_sys(za_ctx* c, int mode, const SweepArgs& a) {
  const CfgArg<double> cfg = make_cfg<double>(c->prob);
  const int nseg = (a.g.nx + XS_CELLS - 1) / XS_CELLS;
  const long long waves = (long long)a.g.ny * nseg;
  const dim3 grid((unsigned)((waves + 3) / 4)), blk(256);
  constexpr int XW = OrderWaves<R>::x;
  if (!general_weights(c->prob) && mode != MODE_FLUX) {
    switch (mode) {
      case MODE_RHS: hipLaunchKernelGGL((k_sweep_x_r<SYS, M, double, MODE_RHS, WV_Z1, R, XW>), grid, blk, 0, c->stream, a, cfg); break;
      case MODE_LX: hipLaunchKernelGGL((k_sweep_x_r<SYS, M, double, MODE_LX, WV_Z1, R, XW>), grid, blk, 0, c->stream, a, cfg); break;
      default: hipLaunchKernelGGL((k_sweep_x_r<SYS, M, double, MODE_STAGE, WV_Z1, R, XW>), grid, blk, 0, c->stream, a, cfg); break;
    }
    return;
  }
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
  constexpr int YW = OrderWaves<R>::y;
  if (!general_weights(c->prob) && mode != MODE_FLUX) {
    if (mode == MODE_RHS)
      hipLaunchKernelGGL((k_sweep_y_r<SYS, M, double, MODE_RHS, WV_Z1, R, YW>), grid, blk, 0, c->stream, a, cfg);
    else
      hipLaunchKernelGGL((k_sweep_y_r<SYS, M, double, MODE_STAGE, WV_Z1, R, YW>), grid, blk, 0, c->stream, a, cfg);
    return;
  }
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

// Resident blocks per CU of the stage y-sweep of this order (for the band
// height); 0 if unknown.
int order_y_blocks_per_cu(const za_problem& p) {
  const void* fn = nullptr;
  const bool gp = general_weights(p);
#define ZA_YFN(R)                                                                                      \
  (p.system == ZA_EULER                                                                                \
       ? (gp ? reinterpret_cast<const void*>(&k_sweep_y_any<SYS_EULER, 4, double, MODE_STAGE, WV_GENERAL, R>) \
             : reinterpret_cast<const void*>(&k_sweep_y_r<SYS_EULER, 4, double, MODE_STAGE, WV_Z1, R, OrderWaves<R>::y>)) \
       : (gp ? reinterpret_cast<const void*>(&k_sweep_y_any<SYS_ADV, 1, double, MODE_STAGE, WV_GENERAL, R>)   \
             : reinterpret_cast<const void*>(&k_sweep_y_r<SYS_ADV, 1, double, MODE_STAGE, WV_Z1, R, OrderWaves<R>::y>)))
  switch (order_of(p)) {
    case 2: fn = ZA_YFN(2); break;
    case 4: fn = ZA_YFN(4); break;
    default: fn = ZA_YFN(5); break;
  }
#undef ZA_YFN
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, 0) != hipSuccess) return 0;
  return n;
}
