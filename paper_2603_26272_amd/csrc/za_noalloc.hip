// za_rhs_noalloc: the right-hand side without a context, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The only device memory the right-hand side needs beyond its input and
// output is the wave-speed reduction: the per-block maxima of the reduction
// pass (at most RED_BLOCKS_MAX blocks, whatever the grid size, since that
// pass strides over the cells) and the control block that carries the
// Lax-Friedrichs speeds to the sweeps.  Both live in `scratch`, a fixed
// device array of this file; each GPU holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in): the device address of each GPU's copy is fetched once
// with hipGetSymbolAddress, with that device current, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "za.h"
#include "za_internal.hpp"

using namespace za;

namespace {

// reduction partials, then the control block at a 256-byte boundary
constexpr size_t kPartDoubles = (size_t)RED_BLOCKS_MAX * NPART;
constexpr size_t kCtlOffset = (kPartDoubles * sizeof(double) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kCtlOffset + 256;
static_assert(sizeof(DevCtl) <= 256, "control block larger than its scratch slot");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

// The device address of this device's copy of `scratch` (looked up once per
// device, with that device current); nullptr if the lookup fails.
static char* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  return g_scratch[dev];
}

extern "C" za_status za_rhs_noalloc(const za_problem* p, const double* q, double* rhs, void* hip_stream) {
  if (!q || !rhs || q == rhs) return ZA_ERR_ARG;
  if (za_validate(p, nullptr) != ZA_OK) return ZA_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ZA_ERR_DEVICE;
  char* base = scratch_on(dev);
  if (!base) return ZA_ERR_DEVICE;
  za_ctx c;   // no workspace: the scratch array stands in for it
  init_shape(&c, p, (hipStream_t)hip_stream);
  if (c.red_blocks > RED_BLOCKS_MAX) return ZA_ERR_ARG;   // the scratch holds RED_BLOCKS_MAX rows
  c.part = reinterpret_cast<double*>(base);
  c.ctl = reinterpret_cast<DevCtl*>(base + kCtlOffset);
  launch_ctl_reset(&c);
  launch_wave(&c, q, FIN_RHS, 0);
  SweepArgs a = base_args(&c);
  a.q = q;
  a.out = rhs;
  launch_x(&c, MODE_RHS, a);
  if (p->dim == 2) {
    a.lx = rhs;
    launch_y(&c, MODE_RHS, a);
  }
  return hipGetLastError() == hipSuccess ? ZA_OK : ZA_ERR_DEVICE;
}
