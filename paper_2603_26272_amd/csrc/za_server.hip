// Continuous-batching server of libza (the za_server_* calls of za.h).
//
// Requests (1D or 2D Euler solves of any size, FP64 or FP32 reconstruction)
// are admitted while a slot is free and their device footprint fits the HBM
// budget, which is one pre-allocated pool sub-allocated first-fit.  Each
// scheduler step advances every admitted request by one SSP-RK3 step: per
// class (dim x precision) one launch per kernel of the step covers the
// blocks of all the class's requests, and each block finds its request in a
// device slot table by binary search over prefix block offsets.  The step of
// a class is a hipGraph captured once per grid capacity (power-of-two block
// counts; surplus blocks exit at once), so admitting or retiring requests
// only rewrites the table.  Classes run on separate streams and overlap.
// Every request keeps its own Lax-Friedrichs speeds, dt and step count, and
// its arithmetic does not depend on the rest of the batch, so a result is
// the same bit for bit alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "za.h"
#include "za_internal.hpp"
#include "za_kernels.hpp"

namespace zs {
using namespace za;

constexpr int MAX_SLOTS = 256;  // per class
constexpr int NCLASS = 4;       // (1D, 2D) x (FP64, FP32 reconstruction)
constexpr int SERVE_YTILE = 8 * YS_ROWS - 1; // default y-sweep rows per block in batches (a whole number of steps)

struct SlotDesc {
  double* st;        // the request's state (Q^n, then the result)
  double* q1;        // RK3 stage states
  double* q2;
  double* lx;        // 2D: x-sweep partial RHS
  double* part;      // wave-speed maxima per stage-kernel block
  DevCtl* ctl;       // the request's control block
  Geom g;
  Phys ph;
  double eps16, eps4, mu0x2;
  int xblocks;       // x-sweep blocks
  int ystrips;       // y-sweep: 64-column strips
  int yblocks;       // y-sweep blocks (strips x tiles)
  int stage_blocks;  // rows of wave-speed maxima the kernel that writes a stage state leaves
  int xl_chunks;     // FP64: chunks per segment of the looped x-sweep
  int ytile;         // 2D: y-sweep rows per block (band height)
};

struct BatchTable {
  int n, xtot, ytot, pad;
  int xoff[MAX_SLOTS + 1];
  int yoff[MAX_SLOTS + 1];
  SlotDesc s[MAX_SLOTS];
};

__device__ __forceinline__ int find_slot(const int* __restrict__ off, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ SweepArgs slot_args(const SlotDesc& d, int stage, bool lx_out) {
  SweepArgs a;
  a.q = stage == 0 ? d.st : (stage == 1 ? d.q1 : d.q2);
  a.qn = d.st;
  a.lx = d.lx;
  a.out = lx_out ? d.lx : (stage == 0 ? d.q1 : (stage == 1 ? d.q2 : d.st));
  a.ctl = d.ctl;
  a.g = d.g;
  a.ph = d.ph;
  a.ca = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
  a.cb = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
  a.check_active = 1;
  a.ytile = d.ytile;
  a.part = d.part;
  a.xl_chunks = d.xl_chunks;
  return a;
}

template <class T>
__device__ __forceinline__ CfgArg<T> slot_cfg(const SlotDesc& d) {
  CfgArg<T> c;
  c.w.eps16 = (T)d.eps16;
  c.w.eps6 = (T)(0.375 * d.eps16);     // 6 eps, rounded once from the exact 16 eps
  c.w.eps6q = (T)(0.09375 * d.eps16);  // 1.5 eps, likewise
  c.w.eps4 = (T)d.eps4;
  c.w.mu0x2 = (T)d.mu0x2;
  c.w.p = T(1);
  c.w.ai = 0;
  c.w.linear = 0;
  c.w.alt_tau = 0;
  c.w.L = T(1);
  c.w.q = T(1);
  c.w.pq = T(1);
  return c;
}

#ifndef ZA_SRV_XS_WAVES
#define ZA_SRV_XS_WAVES 3   // the slot lookup costs registers: four waves per SIMD would spill
#endif
template <int M, class T>
__global__ __launch_bounds__(256, ZA_SRV_XS_WAVES) void kb_sweep_x(const BatchTable* __restrict__ tab, int stage) {
  const int b = blockIdx.x;
  if (b >= tab->xtot) return;
  const int s = find_slot(tab->xoff, tab->n, b);
  const SlotDesc& d = tab->s[s];
  const SweepArgs a = slot_args(d, stage, M == 4);
  const CfgArg<T> cfg = slot_cfg<T>(d);
  if (M == 4)
    sweep_x_body<SYS_EULER, M, T, MODE_LX, WV_Z1>(a, cfg, b - tab->xoff[s]);
  else
    sweep_x_body<SYS_EULER, M, T, MODE_STAGE, WV_Z1>(a, cfg, b - tab->xoff[s]);
}

// FP64 classes: the looped x-sweep (2D: partial stage; 1D: the whole stage
// and one row of wave-speed maxima per wavefront).
template <int M>
__global__ __launch_bounds__(256, 3) void kb_sweep_xl(const BatchTable* __restrict__ tab, int stage) {
  const int b = blockIdx.x;
  if (b >= tab->xtot) return;
  const int s = find_slot(tab->xoff, tab->n, b);
  const SlotDesc& d = tab->s[s];
  const SweepArgs a = slot_args(d, stage, M == 4);
  const CfgArg<double> cfg = slot_cfg<double>(d);
  sweep_xl_body<SYS_EULER, M, WV_Z1, M == 4 ? MODE_LX : MODE_STAGE>(a, cfg, b - tab->xoff[s]);
}

template <class T>
__global__ __launch_bounds__(256, ZA_YS_WAVES) void kb_sweep_y(const BatchTable* __restrict__ tab, int stage) {
  const int b = blockIdx.x;
  if (b >= tab->ytot) return;
  const int s = find_slot(tab->yoff, tab->n, b);
  const SlotDesc& d = tab->s[s];
  const SweepArgs a = slot_args(d, stage, false);
  const CfgArg<T> cfg = slot_cfg<T>(d);
  const int local = b - tab->yoff[s];
  sweep_y_body<SYS_EULER, 4, T, MODE_STAGE, WV_Z1>(a, cfg, local % d.ystrips,
                                                   local / d.ystrips, d.ystrips);
}

__global__ __launch_bounds__(64) void kb_final(const BatchTable* __restrict__ tab, int kind, int dim) {
  const int s = blockIdx.x;
  if (s >= tab->n) return;
  const SlotDesc& d = tab->s[s];
  wave_final_body(d.part, d.stage_blocks, d.ctl, d.g, d.ph, dim, kind, SYS_EULER);
}

__global__ __launch_bounds__(64) void kb_step_end(const BatchTable* __restrict__ tab) {
  const int s = blockIdx.x;
  if (s >= tab->n) return;
  step_end_body(tab->s[s].ctl);
}

__global__ void k_ctl_set(DevCtl* ctl, DevCtl v) {
  if (threadIdx.x == 0) *ctl = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Pool {  // first-fit sub-allocation of [0, cap), 256-byte granules
  std::map<size_t, size_t> free_;
  void init(size_t cap) { free_.clear(); free_[0] = cap; }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, base = it->first + n;
        free_.erase(it);
        if (rest) free_[base] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  za_req_id id = 0;
  za_problem prob;
  int cls = 0, m = 1;
  size_t ncell = 0;
  std::vector<double> q0;           // initial state until its upload (no pinned space)
  std::unique_ptr<double[]> qout;   // final state after its download (no pinned space)
  double* h_in = nullptr;           // initial state in the pinned staging pool
  double* h_out = nullptr;          // final state in the pinned staging pool
  size_t h_in_off = 0, h_out_off = 0;
  bool xfer_ok = false;             // result of the last transfer
  int64_t n_steps = 0;
  int64_t t_arr = 0, t_adm = 0, t_fin = 0;
  int status = ZA_OK;
  bool admitted = false, done = false;
  int slot = -1;           // fixed control-block index in its class
  size_t off = 0, bytes = 0;
  SlotDesc desc;
  int64_t steps = 0, interfaces = 0;
  int64_t launched = 0;    // RK3 steps enqueued since admission
};

// One burst of RK3 steps of a class in flight: the requests it advanced, the
// host buffers it used (table upload, control-block mirror) and the event
// recorded after its mirror copy.
struct Burst {
  int buf = 0;
  hipEvent_t ev = nullptr;
  std::vector<Req*> members;
};

// A transfer for the transfer thread: the initial state of an admitted
// request (up) or the final state of a finished one.
struct XJob {
  Req* r;
  bool up;
};

// RK3 steps of a class per burst: SERVE_MAX_BURST, or fewer when every
// active request needs fewer.  A request that reaches its step count stops
// on the device (its control block turns inactive and its blocks exit at
// once), so it ends mid-burst and never waits for the others.  Each class
// keeps SERVE_DEPTH bursts queued on its stream, so the GPU works on the
// next burst while the host retires and admits requests.
constexpr int SERVE_MAX_BURST = 8;
constexpr int SERVE_DEPTH = 2;       // default; ZA_SRV_DEPTH overrides (1 .. SERVE_DEPTH_MAX)
constexpr int SERVE_DEPTH_MAX = 4;

static int class_of(const za_problem& p) { return (p.dim == 2 ? 2 : 0) + (p.precision == ZA_FP32_RECON ? 1 : 0); }
static int ncomp(const za_problem& p) { return p.dim == 1 ? 3 : 4; }

struct GraphKey {
  int xcap, ycap, ncap;
  bool operator<(const GraphKey& o) const {
    return xcap != o.xcap ? xcap < o.xcap : (ycap != o.ycap ? ycap < o.ycap : ncap < o.ncap);
  }
};

struct Class {
  hipStream_t stream = nullptr;
  BatchTable* dtab = nullptr;
  BatchTable* htab[SERVE_DEPTH_MAX] = {};   // pinned: the table each queued burst uploaded
  DevCtl* dctl = nullptr;               // MAX_SLOTS control blocks
  DevCtl* hctl[SERVE_DEPTH_MAX] = {};       // pinned: control blocks after each queued burst
  hipEvent_t ev[SERVE_DEPTH_MAX] = {};
  std::deque<Burst> inflight;           // oldest first
  std::vector<Req*> active;
  std::vector<int> free_slots;
  bool dirty = true;                    // the device table lags behind `active`
  std::map<GraphKey, hipGraphExec_t> graphs;
  int64_t stat_bursts = 0, stat_steps = 0, stat_members = 0;   // ZA_SRV_STATS=1 prints them at destroy
};

}  // namespace zs

using namespace zs;

struct za_server {
  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  char* pool_base = nullptr;
  Pool pool;
  Class cls[NCLASS];
  std::deque<Req*> waiting;
  std::map<za_req_id, std::unique_ptr<Req>> reqs;
  hipStream_t xfer = nullptr;     // uploads and result downloads, beside the compute streams
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_xfer;
  std::thread th, xth;            // scheduler, transfers
  bool stop = false, xstop = false;
  std::deque<XJob> xjobs;         // transfers queued for xth
  int64_t xpending = 0;           // transfers queued or running
  std::vector<Req*> uploaded;     // uploads done, to be started by the scheduler
  int admitting = 0;              // admitted requests not yet started
  char* hpin = nullptr;           // pinned staging pool for uploads and results
  Pool hpool;
  za_req_id next_id = 1;
  int64_t in_flight = 0;   // submitted and not finished
  std::string err;
  // host-side fault injection for tests of the failure path
  // (ZA_SRV_FAIL_BURST=k: the k-th burst launch reports a launch error)
  int64_t fail_burst = 0, bursts = 0;
  // (ZA_SRV_FAIL_XFER=k: the k-th upload or download reports a copy error)
  int64_t fail_xfer = 0, xfers = 0;
  bool graphs = true;   // replay a captured graph per class step (ZA_SRV_GRAPHS=0: direct launches)
  int64_t max_burst = SERVE_MAX_BURST;   // ZA_SRV_BURST overrides (1 .. 64)
  int depth = SERVE_DEPTH;               // bursts queued per class
};

constexpr long long kServeMinWaves = 3072;   // 3 per SIMD of a 256-CU device

// Chunks per segment of the looped x-sweep, which FP64 requests always use
// (0 for FP32 reconstruction: the one-shot sweep), fixed at admission (its
// wave-speed rows depend on it in 1D).  2D: the count that minimises the
// work of a row, segments x (chunks + 0.15 for a segment's start), since a
// row of n cells takes ceil(n / (64 nc - 1)) segments and a last segment of a
// few cells costs as much as a full one (n = 1024: 3 chunks, 6 segments,
// instead of 4 chunks, 5 segments), among the counts that leave a request
// at least kServeMinWaves wavefronts (its latency when alone).  1D: up to
// 4 chunks, which keeps many
// wavefronts per request.  ZA_SRV_XL_CHUNKS in the environment forces a
// value, clamped to 1 .. 64.
static int serve_xl_chunks(const za_problem& p) {
  if (p.precision != ZA_FP64) return 0;
  if (const char* e = std::getenv("ZA_SRV_XL_CHUNKS")) return std::max(1, std::min(std::atoi(e), 64));
  if (p.dim == 1) return std::max(1, std::min(4, p.nx / 2048));
  int best = 1;
  double best_cost = -1.0;
  for (int nc = 1; nc <= 16; ++nc) {
    const long long seg = 64LL * nc - 1;
    const long long segs = (p.nx + seg - 1) / seg;
    // a request alone still fills three wavefronts per SIMD where it can
    if (nc > 1 && (long long)p.ny * segs < kServeMinWaves) break;
    const double cost = (double)segs * (nc + 0.15);
    if (best_cost < 0.0 || cost < best_cost) { best_cost = cost; best = nc; }
    if (seg >= p.nx) break;   // one segment per row from here on
  }
  return best;
}

// Rows per y-sweep block of a 2D request, fixed at admission:
// SERVE_YTILE, or ZA_SRV_YTILE from the environment (rounded to a whole
// number of YS_ROWS-row steps, at least one).
static int serve_ytile(const za_problem& p) {
  (void)p;
  if (const char* e = std::getenv("ZA_SRV_YTILE")) {
    const int v = std::max(1, std::atoi(e) / YS_ROWS);
    return YS_ROWS * std::min(v, 256) - 1;
  }
  return SERVE_YTILE;
}

static size_t footprint(const za_problem& p, int* stage_blocks, int* xblocks, int* ystrips, int* yblocks,
                        int* xl_chunks, int* ytile) {
  const int m = ncomp(p);
  const size_t S = (size_t)m * p.nx * p.ny * sizeof(double);
  *xl_chunks = serve_xl_chunks(p);
  *ytile = serve_ytile(p);
  const long long xw = *xl_chunks > 0 ? xl_waves(p.nx, p.ny, *xl_chunks)
                                      : (long long)p.ny * ((p.nx + XS_CELLS - 1) / XS_CELLS);
  *xblocks = (int)((xw + 3) / 4);
  if (p.dim == 2) {
    *ystrips = (p.nx + 63) / 64;
    *yblocks = *ystrips * ((p.ny + *ytile - 1) / *ytile);
    *stage_blocks = *yblocks;
  } else {
    *ystrips = 0;
    *yblocks = 0;
    *stage_blocks = *xl_chunks > 0 ? (int)xw : *xblocks;
  }
  const size_t part = ((size_t)*stage_blocks * NPART * sizeof(double) + 255) & ~size_t(255);
  return (p.dim == 2 ? 4 : 3) * ((S + 255) & ~size_t(255)) + part;
}

static int pow2_cap(int n, int lo) {
  int c = lo;
  while (c < n) c <<= 1;
  return c;
}

// Launch one RK3 step of a class (captured into a graph per capacity) for
// the table h, which the device table holds by the time the step runs.
static void enqueue_class_step(Class& C, int c, const GraphKey& key) {
  const bool two_d = c >= 2, fp32 = (c & 1) != 0;
  for (int s = 0; s < 3; ++s) {
    hipLaunchKernelGGL(kb_final, dim3(key.ncap), dim3(64), 0, C.stream, C.dtab, s == 0 ? FIN_STAGE0 : FIN_STAGEK,
                       two_d ? 2 : 1);
    if (two_d) {
      if (fp32) {
        hipLaunchKernelGGL((kb_sweep_x<4, float>), dim3(key.xcap), dim3(256), 0, C.stream, C.dtab, s);
        hipLaunchKernelGGL((kb_sweep_y<float>), dim3(key.ycap), dim3(256), 0, C.stream, C.dtab, s);
      } else {
        hipLaunchKernelGGL((kb_sweep_xl<4>), dim3(key.xcap), dim3(256), 0, C.stream, C.dtab, s);
        hipLaunchKernelGGL((kb_sweep_y<double>), dim3(key.ycap), dim3(256), 0, C.stream, C.dtab, s);
      }
    } else {
      if (fp32)
        hipLaunchKernelGGL((kb_sweep_x<3, float>), dim3(key.xcap), dim3(256), 0, C.stream, C.dtab, s);
      else
        hipLaunchKernelGGL((kb_sweep_xl<3>), dim3(key.xcap), dim3(256), 0, C.stream, C.dtab, s);
    }
  }
  hipLaunchKernelGGL(kb_step_end, dim3(key.ncap), dim3(64), 0, C.stream, C.dtab);
}

static hipError_t class_step(za_server* sv, int c, const BatchTable& h) {
  Class& C = sv->cls[c];
  const bool two_d = c >= 2;
  GraphKey key{pow2_cap(h.xtot, 64), two_d ? pow2_cap(h.ytot, 64) : 0, pow2_cap(h.n, 8)};
  if (!sv->graphs) {   // direct launches: exact grids
    enqueue_class_step(C, c, GraphKey{std::max(h.xtot, 1), two_d ? std::max(h.ytot, 1) : 0, std::max(h.n, 1)});
    return hipGetLastError();
  }
  auto it = C.graphs.find(key);
  if (it == C.graphs.end()) {
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(C.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    enqueue_class_step(C, c, key);
    e = hipStreamEndCapture(C.stream, &g);
    if (e != hipSuccess) return e;
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    it = C.graphs.emplace(key, ex).first;
  }
  return hipGraphLaunch(it->second, C.stream);
}

static void rebuild_table(const Class& C, BatchTable& h) {
  h.n = (int)C.active.size();
  int x = 0, y = 0;
  for (int i = 0; i < h.n; ++i) {
    h.s[i] = C.active[i]->desc;
    h.xoff[i] = x;
    h.yoff[i] = y;
    x += h.s[i].xblocks;
    y += h.s[i].yblocks;
  }
  h.xoff[h.n] = x;
  h.yoff[h.n] = y;
  h.xtot = x;
  h.ytot = y;
}

// Bytes of one state of r in the pinned staging pool.
static size_t host_bytes(const Req* r) { return (r->m * r->ncell * sizeof(double) + 255) & ~size_t(255); }

// Take r out of its class (lock held): its slot is free and no later burst
// table holds it; its pool memory stays until complete_req.
static void retire_req(za_server* sv, Req* r) {
  Class& C = sv->cls[r->cls];
  if (r->slot >= 0) C.free_slots.push_back(r->slot);
  r->slot = -1;
  C.active.erase(std::remove(C.active.begin(), C.active.end(), r), C.active.end());
  for (Burst& b : C.inflight) b.members.erase(std::remove(b.members.begin(), b.members.end(), r), b.members.end());
  C.dirty = true;
}

// Mark r finished with status st (its result, if any, already in r->qout)
// and release its pool memory (lock held).
static void complete_req(za_server* sv, Req* r, int st) {
  if (r->done) return;
  r->status = st;
  if (r->h_in) sv->hpool.release(r->h_in_off, host_bytes(r));
  r->h_in = nullptr;
  if (r->bytes) sv->pool.release(r->off, r->bytes);
  r->bytes = 0;
  r->done = true;
  r->t_fin = now_ns();
  sv->in_flight--;
  std::vector<double>().swap(r->q0);
}

static void finish_req(za_server* sv, Req* r, int st) {
  if (r->done) return;
  retire_req(sv, r);
  complete_req(sv, r, st);
}

// A device failure in class c: drain its stream and end every request it
// holds with ZA_ERR_DEVICE (lock held).
static void fail_class(za_server* sv, int c, const char* what) {
  Class& C = sv->cls[c];
  sv->err = what;
  (void)hipStreamSynchronize(C.stream);
  (void)hipGetLastError();
  C.inflight.clear();
  while (!C.active.empty()) finish_req(sv, C.active.back(), ZA_ERR_DEVICE);
  sv->cv_done.notify_all();
}

// Admit waiting requests that fit (first fit in arrival order, lock held):
// pool space and a slot are taken here, and the initial state is queued for
// the transfer thread (activate_uploaded starts the request afterwards).
static void admit(za_server* sv) {
  int total = sv->admitting;   // admitted, upload not yet done
  for (int c = 0; c < NCLASS; ++c) total += (int)sv->cls[c].active.size();
  std::vector<Req*> picked;
  for (auto it = sv->waiting.begin(); it != sv->waiting.end();) {
    Req* r = *it;
    Class& C = sv->cls[r->cls];
    if (total >= sv->max_slots) break;
    if (C.free_slots.empty()) { ++it; continue; }
    int sb, xb, ys, yb, xc, yt;
    const size_t need = footprint(r->prob, &sb, &xb, &ys, &yb, &xc, &yt);
    size_t off;
    if (!sv->pool.alloc(need, &off)) { ++it; continue; }
    r->off = off;
    r->bytes = need;
    r->slot = C.free_slots.back();
    C.free_slots.pop_back();
    const size_t S = ((r->m * r->ncell * sizeof(double)) + 255) & ~size_t(255);
    char* base = sv->pool_base + off;
    SlotDesc& d = r->desc;
    std::memset(&d, 0, sizeof(d));
    d.st = (double*)base;
    d.q1 = (double*)(base + S);
    d.q2 = (double*)(base + 2 * S);
    d.lx = r->prob.dim == 2 ? (double*)(base + 3 * S) : nullptr;
    d.part = (double*)(base + (r->prob.dim == 2 ? 4 : 3) * S);
    d.ctl = C.dctl + r->slot;
    const za_problem& p = r->prob;
    d.g.nx = p.nx; d.g.ny = p.ny; d.g.bc_x = p.bc_x; d.g.bc_y = p.bc_y;
    d.g.dx = (p.xhi - p.xlo) / p.nx;
    d.g.dy = p.dim == 2 ? (p.yhi - p.ylo) / p.ny : 1.0;
    d.g.inv_dx = 1.0 / d.g.dx;
    d.g.inv_dy = 1.0 / d.g.dy;
    d.ph.gamma = p.gamma; d.ph.gm1 = p.gamma - 1.0;
    d.ph.adv[0] = p.adv_speed[0]; d.ph.adv[1] = p.adv_speed[1];
    d.ph.cfl = p.cfl; d.ph.dt_rule = p.dt_rule; d.ph.lf_scalar = p.lf == ZA_LF_SCALAR ? 1 : 0;
    d.ph.pp = 0;   // requests with the limiter are not admitted
    d.eps16 = 16.0 * p.eps; d.eps4 = 4.0 * p.eps; d.mu0x2 = 2.0 * p.mu0;
    d.xblocks = xb; d.ystrips = ys; d.yblocks = yb; d.stage_blocks = sb; d.xl_chunks = xc; d.ytile = yt;
    picked.push_back(r);
    ++total;
    it = sv->waiting.erase(it);
  }
  for (Req* r : picked) {
    sv->xjobs.push_back({r, true});
    ++sv->xpending;
    ++sv->admitting;
  }
  if (!picked.empty()) sv->cv_xfer.notify_one();
}

// Requests whose upload finished (lock held): enqueue their control block
// and the wave speeds of Q^0 on the class stream and make them active.
static void activate_uploaded(za_server* sv) {
  for (Req* r : sv->uploaded) {
    Class& C = sv->cls[r->cls];
    --sv->admitting;
    r->admitted = true;
    r->t_adm = now_ns();
    if (!r->xfer_ok) {
      sv->err = "request upload failed";
      finish_req(sv, r, ZA_ERR_DEVICE);
      sv->cv_done.notify_all();
      continue;
    }
    const SlotDesc& d = r->desc;
    DevCtl v;
    std::memset(&v, 0, sizeof(v));
    v.t_final = std::numeric_limits<double>::infinity();
    v.dt_min = std::numeric_limits<double>::infinity();
    v.bad_step = -1;
    v.active = 1;
    v.max_steps = r->n_steps;
    // stream order puts this after the queued bursts, which may still see
    // the slot's previous request (inactive) in their tables
    hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(64), 0, C.stream, d.ctl, v);
    if (r->prob.dim == 2)
      hipLaunchKernelGGL((k_wave_partial<SYS_EULER, 4>), dim3(d.stage_blocks), dim3(256), 0, C.stream, d.st,
                         r->ncell, d.ph, d.ctl, 0, d.part);
    else
      hipLaunchKernelGGL((k_wave_partial<SYS_EULER, 3>), dim3(d.stage_blocks), dim3(256), 0, C.stream, d.st,
                         r->ncell, d.ph, d.ctl, 0, d.part);
    if (hipGetLastError() != hipSuccess) {
      sv->err = "request start failed";
      finish_req(sv, r, ZA_ERR_DEVICE);
      sv->cv_done.notify_all();
      continue;
    }
    C.active.push_back(r);
    C.dirty = true;
    std::vector<double>().swap(r->q0);
  }
  sv->uploaded.clear();
}

// The transfer thread: uploads of admitted requests and downloads of
// finished ones on the transfer stream, so that the scheduler keeps every
// class's bursts queued meanwhile.  It takes every queued transfer at once,
// issues the copies and waits once; copies between the device and the
// pinned staging pool are plain DMA (the pageable fallback, when the pool is
// full, is staged by the runtime).  An upload hands the request back to the
// scheduler; a download completes it.
static void xfer_worker(za_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  std::vector<XJob> batch;
  while (true) {
    sv->cv_xfer.wait(lk, [&] { return sv->xstop || !sv->xjobs.empty(); });
    if (sv->xjobs.empty()) break;   // xstop and nothing left
    batch.assign(sv->xjobs.begin(), sv->xjobs.end());
    sv->xjobs.clear();
    for (const XJob& j : batch) {   // pinned space for the results
      Req* r = j.r;
      size_t off;
      if (!j.up && sv->hpool.alloc(host_bytes(r), &off)) {
        r->h_out = (double*)(sv->hpin + off);
        r->h_out_off = off;
      }
    }
    lk.unlock();
    std::vector<char> ok(batch.size(), 1);
    for (size_t k = 0; k < batch.size(); ++k) {
      Req* r = batch[k].r;
      const size_t n = r->m * r->ncell;
      if (sv->fail_xfer > 0 && ++sv->xfers == sv->fail_xfer) {
        ok[k] = 0;   // injected: this transfer reports a failure, no copy is made
        continue;
      }
      if (batch[k].up) {
        const double* src = r->h_in ? r->h_in : r->q0.data();
        ok[k] = hipMemcpyAsync(r->desc.st, src, n * sizeof(double), hipMemcpyHostToDevice, sv->xfer) == hipSuccess;
      } else {
        double* dst = r->h_out;
        if (!dst) {
          r->qout.reset(new double[n]);
          dst = r->qout.get();
        }
        ok[k] = hipMemcpyAsync(dst, r->desc.st, n * sizeof(double), hipMemcpyDeviceToHost, sv->xfer) == hipSuccess;
      }
    }
    const bool synced = hipStreamSynchronize(sv->xfer) == hipSuccess;
    lk.lock();
    bool any_up = false, any_down = false;
    for (size_t k = 0; k < batch.size(); ++k) {
      Req* r = batch[k].r;
      --sv->xpending;
      r->xfer_ok = synced && ok[k];
      if (batch[k].up) {
        if (r->h_in) sv->hpool.release(r->h_in_off, host_bytes(r));
        r->h_in = nullptr;
        sv->uploaded.push_back(r);
        any_up = true;
      } else {
        if (!r->xfer_ok) sv->err = "result download failed";
        complete_req(sv, r, r->xfer_ok ? r->status : (int)ZA_ERR_DEVICE);
        any_down = true;
      }
    }
    if (any_up) sv->cv_work.notify_one();
    if (any_down) sv->cv_done.notify_all();
  }
}

// Queue one burst of RK3 steps of class c (lock held): upload the table if
// the active set changed, launch the steps, copy the control blocks back
// and record an event.
static void launch_burst(za_server* sv, int c) {
  Class& C = sv->cls[c];
  int buf = 0;
  if (!C.inflight.empty()) buf = (C.inflight.back().buf + 1) % sv->depth;   // fewer than depth in flight
  BatchTable& h = *C.htab[buf];
  rebuild_table(C, h);
  if (C.dirty) {
    if (hipMemcpyAsync(C.dtab, &h, sizeof(BatchTable), hipMemcpyHostToDevice, C.stream) != hipSuccess) {
      fail_class(sv, c, "table upload failed");
      return;
    }
    C.dirty = false;
  }
  int64_t burst = 1;
  for (const Req* r : C.active) burst = std::max(burst, r->n_steps - r->launched);
  burst = std::min<int64_t>(burst, sv->max_burst);
  ++sv->bursts;
  if (sv->fail_burst > 0 && sv->bursts == sv->fail_burst) {
    fail_class(sv, c, "graph launch failed (injected)");
    return;
  }
  for (int64_t k = 0; k < burst; ++k) {
    if (class_step(sv, c, h) != hipSuccess) {
      fail_class(sv, c, "graph launch failed");
      return;
    }
  }
  for (Req* r : C.active) r->launched += burst;
  C.stat_bursts++;
  C.stat_steps += burst;
  C.stat_members += (int64_t)C.active.size() * burst;
  if (hipMemcpyAsync(C.hctl[buf], C.dctl, MAX_SLOTS * sizeof(DevCtl), hipMemcpyDeviceToHost, C.stream) != hipSuccess ||
      hipEventRecord(C.ev[buf], C.stream) != hipSuccess) {
    fail_class(sv, c, "control block copy failed");
    return;
  }
  Burst b;
  b.buf = buf;
  b.ev = C.ev[buf];
  b.members = C.active;
  C.inflight.push_back(std::move(b));
}

// The requests a completed burst finished (lock held).
static void collect_finished(za_server* sv, int c, const Burst& b, std::vector<Req*>* out) {
  const DevCtl* hc = sv->cls[c].hctl[b.buf];
  for (Req* r : b.members) {
    const DevCtl& h = hc[r->slot];
    if (h.active) continue;
    r->steps = h.steps;
    const long long irs = r->prob.dim == 2 ? (long long)(r->prob.nx + 1) * r->prob.ny +
                                                 (long long)r->prob.nx * (r->prob.ny + 1)
                                           : (long long)(r->prob.nx + 1);
    r->interfaces = 3 * irs * h.steps;
    r->status = h.bad ? ZA_ERR_NONFINITE : ZA_OK;
    out->push_back(r);
  }
}

static void scheduler(za_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  std::vector<Req*> fin;
  while (true) {
    admit(sv);
    activate_uploaded(sv);
    bool any = sv->xpending > 0;
    for (int c = 0; c < NCLASS; ++c) {
      Class& C = sv->cls[c];
      if (!C.active.empty() && (int)C.inflight.size() < sv->depth) launch_burst(sv, c);
      any = any || !C.active.empty() || !C.inflight.empty();
    }
    if (!any) {
      if (sv->stop) break;
      sv->cv_work.wait(lk, [&] { return sv->stop || !sv->waiting.empty() || !sv->uploaded.empty(); });
      continue;
    }
    // completed bursts, oldest first per class
    bool progressed = false;
    fin.clear();
    for (int c = 0; c < NCLASS; ++c) {
      Class& C = sv->cls[c];
      while (!C.inflight.empty()) {
        const hipError_t q = hipEventQuery(C.inflight.front().ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          fail_class(sv, c, "burst failed");
          break;
        }
        collect_finished(sv, c, C.inflight.front(), &fin);
        C.inflight.pop_front();
        progressed = true;
      }
    }
    if (!fin.empty()) {
      // out of their classes now; the transfer thread copies the results
      // out and completes them (a request leaves the device only then)
      std::sort(fin.begin(), fin.end());
      fin.erase(std::unique(fin.begin(), fin.end()), fin.end());
      for (Req* r : fin) {
        retire_req(sv, r);
        sv->xjobs.push_back({r, false});
        ++sv->xpending;
      }
      sv->cv_xfer.notify_one();
    }
    if (!progressed && sv->uploaded.empty()) {
      // nothing finished yet: sleep briefly (a submission or an upload wakes us)
      sv->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

extern "C" {

za_status za_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t device, za_server** out) {
  if (!out) return ZA_ERR_ARG;
  *out = nullptr;
  if (hbm_budget_bytes < (1u << 20) || max_slots < 1 || max_slots > MAX_SLOTS) return ZA_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ZA_ERR_ARG;
  auto sv = std::make_unique<za_server>();
  // on failure, free whatever was created so far (no scheduler thread yet)
  auto fail = [&](za_status st) { za_server_destroy(sv.release()); return st; };
  sv->budget = hbm_budget_bytes;
  sv->max_slots = max_slots;
  sv->device = device;
  if (const char* e = std::getenv("ZA_SRV_FAIL_BURST")) sv->fail_burst = std::atoll(e);
  if (const char* e = std::getenv("ZA_SRV_FAIL_XFER")) sv->fail_xfer = std::atoll(e);
  if (const char* e = std::getenv("ZA_SRV_GRAPHS")) sv->graphs = std::atoi(e) != 0;
  if (const char* e = std::getenv("ZA_SRV_BURST")) sv->max_burst = std::max(1, std::min(std::atoi(e), 64));
  if (const char* e = std::getenv("ZA_SRV_DEPTH")) sv->depth = std::max(1, std::min(std::atoi(e), SERVE_DEPTH_MAX));
  if (hipSetDevice(device) != hipSuccess) return fail(ZA_ERR_DEVICE);
  void* p = nullptr;
  if (hipMalloc(&p, hbm_budget_bytes) != hipSuccess) return fail(ZA_ERR_NOMEM);
  sv->pool_base = (char*)p;
  sv->pool.init(hbm_budget_bytes);
  {
    // pinned staging: as large as the device budget, at most 1 GiB
    // (ZA_SRV_PINNED_MB overrides; 0: none).  If the host cannot pin that
    // much, halve it down to 16 MiB, else run without: requests that find no
    // pinned space pass through pageable memory.
    size_t hb = std::min<size_t>(hbm_budget_bytes, size_t(1) << 30);
    if (const char* e = std::getenv("ZA_SRV_PINNED_MB")) hb = (size_t)std::max(0LL, std::atoll(e)) << 20;
    while (hb >= (size_t(16) << 20) && hipHostMalloc(&p, hb, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      hb /= 2;
    }
    if (hb >= (size_t(16) << 20) || (hb > 0 && hipHostMalloc(&p, hb, hipHostMallocDefault) == hipSuccess)) {
      sv->hpin = (char*)p;
      sv->hpool.init(hb);
    } else {
      (void)hipGetLastError();
      sv->hpool.init(0);
    }
  }
  // non-blocking streams: nothing here waits on the null stream
  if (hipStreamCreateWithFlags(&sv->xfer, hipStreamNonBlocking) != hipSuccess) return fail(ZA_ERR_DEVICE);
  for (int c = 0; c < NCLASS; ++c) {
    Class& C = sv->cls[c];
    if (hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking) != hipSuccess) return fail(ZA_ERR_DEVICE);
    if (hipMalloc(&p, sizeof(BatchTable)) != hipSuccess) return fail(ZA_ERR_NOMEM);
    C.dtab = (BatchTable*)p;
    if (hipMalloc(&p, MAX_SLOTS * sizeof(DevCtl)) != hipSuccess) return fail(ZA_ERR_NOMEM);
    C.dctl = (DevCtl*)p;
    for (int b = 0; b < SERVE_DEPTH_MAX; ++b) {
      if (hipHostMalloc(&p, sizeof(BatchTable), hipHostMallocDefault) != hipSuccess) return fail(ZA_ERR_NOMEM);
      C.htab[b] = (BatchTable*)p;
      std::memset(C.htab[b], 0, sizeof(BatchTable));
      if (hipHostMalloc(&p, MAX_SLOTS * sizeof(DevCtl), hipHostMallocDefault) != hipSuccess) return fail(ZA_ERR_NOMEM);
      C.hctl[b] = (DevCtl*)p;
      std::memset(C.hctl[b], 0, MAX_SLOTS * sizeof(DevCtl));
      if (hipEventCreateWithFlags(&C.ev[b], hipEventDisableTiming) != hipSuccess) return fail(ZA_ERR_DEVICE);
    }
    for (int s = MAX_SLOTS - 1; s >= 0; --s) C.free_slots.push_back(s);
    if (hipMemcpy(C.dtab, C.htab[0], sizeof(BatchTable), hipMemcpyHostToDevice) != hipSuccess) return fail(ZA_ERR_DEVICE);
  }
  za_server* raw = sv.release();
  raw->xth = std::thread(xfer_worker, raw);
  raw->th = std::thread(scheduler, raw);
  *out = raw;
  return ZA_OK;
}

za_status za_server_submit(za_server* sv, const za_problem* p, const double* q0, int64_t n_steps, za_req_id* id) {
  if (!sv || !p || !q0 || !id || n_steps < 1) return ZA_ERR_ARG;
  std::string why;
  {
    const za_status vs = za_validate(p, &why);
    if (vs != ZA_OK) return vs;
  }
  // batches run the paper's weights (Z type, p = 1, mu = 1) on the Euler equations
  if (p->system != ZA_EULER || general_weights(*p) || order_of(*p) != 3 || p->pp_limiter)
    return ZA_ERR_UNSUPPORTED;
  int sb, xb, ys, yb, xc, yt;
  if (footprint(*p, &sb, &xb, &ys, &yb, &xc, &yt) > sv->budget) return ZA_ERR_NOMEM;
  auto r = std::make_unique<Req>();
  r->prob = *p;
  r->cls = class_of(*p);
  r->m = ncomp(*p);
  r->ncell = (size_t)p->nx * p->ny;
  r->n_steps = n_steps;
  {
    size_t off;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->hpool.alloc(host_bytes(r.get()), &off)) {
      r->h_in = (double*)(sv->hpin + off);
      r->h_in_off = off;
    }
  }
  // the copy runs with the lock released; the request is not queued yet
  if (r->h_in) std::memcpy(r->h_in, q0, r->m * r->ncell * sizeof(double));
  else r->q0.assign(q0, q0 + r->m * r->ncell);
  r->t_arr = now_ns();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      if (r->h_in) sv->hpool.release(r->h_in_off, host_bytes(r.get()));
      return ZA_ERR_ARG;
    }
    r->id = sv->next_id++;
    *id = r->id;
    sv->waiting.push_back(r.get());
    sv->reqs.emplace(r->id, std::move(r));
    sv->in_flight++;
  }
  sv->cv_work.notify_one();
  return ZA_OK;
}

za_status za_server_poll(za_server* sv, za_req_id id, int32_t* done, double* q_out, za_req_stats* st) {
  if (!sv || !done) return ZA_ERR_ARG;
  std::unique_ptr<Req> own;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return ZA_ERR_ARG;
    Req* r = it->second.get();
    *done = r->done ? 1 : 0;
    if (st) {
      st->arrival_ns = r->t_arr;
      st->admit_ns = r->t_adm;
      st->finish_ns = r->t_fin;
      st->steps = r->steps;
      st->interfaces = r->interfaces;
      st->status = r->status;
    }
    if (!(r->done && q_out)) return r->done ? (za_status)r->status : ZA_OK;
    own = std::move(it->second);   // the result is copied with the lock released
    sv->reqs.erase(it);
  }
  const size_t n = own->m * own->ncell;
  if (own->h_out) {
    std::memcpy(q_out, own->h_out, n * sizeof(double));
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->hpool.release(own->h_out_off, host_bytes(own.get()));
  } else if (own->qout) {
    std::memcpy(q_out, own->qout.get(), n * sizeof(double));
  }
  return (za_status)own->status;
}

za_status za_server_drain(za_server* sv) {
  if (!sv) return ZA_ERR_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->in_flight == 0; });
  return sv->err.empty() ? ZA_OK : ZA_ERR_DEVICE;
}

za_status za_server_destroy(za_server* sv) {
  if (!sv) return ZA_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->waiting.clear();
  }
  sv->cv_work.notify_all();
  if (sv->th.joinable()) sv->th.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->xstop = true;
  }
  sv->cv_xfer.notify_all();
  if (sv->xth.joinable()) sv->xth.join();
  if (const char* e = std::getenv("ZA_SRV_STATS")) {
    if (std::atoi(e) != 0) {
      for (int c = 0; c < NCLASS; ++c) {
        const Class& C = sv->cls[c];
        std::fprintf(stderr, "za_server class %d: %lld bursts, %.2f steps per burst, %.2f requests per step\n", c,
                     (long long)C.stat_bursts, C.stat_bursts ? (double)C.stat_steps / C.stat_bursts : 0.0,
                     C.stat_steps ? (double)C.stat_members / C.stat_steps : 0.0);
      }
    }
  }
  for (int c = 0; c < NCLASS; ++c) {
    Class& C = sv->cls[c];
    if (C.stream) (void)hipStreamSynchronize(C.stream);
    for (auto& kv : C.graphs) (void)hipGraphExecDestroy(kv.second);
    if (C.dtab) (void)hipFree(C.dtab);
    if (C.dctl) (void)hipFree(C.dctl);
    for (int b = 0; b < SERVE_DEPTH_MAX; ++b) {
      if (C.htab[b]) (void)hipHostFree(C.htab[b]);
      if (C.hctl[b]) (void)hipHostFree(C.hctl[b]);
      if (C.ev[b]) (void)hipEventDestroy(C.ev[b]);
    }
    if (C.stream) (void)hipStreamDestroy(C.stream);
  }
  if (sv->xfer) {
    (void)hipStreamSynchronize(sv->xfer);
    (void)hipStreamDestroy(sv->xfer);
  }
  if (sv->pool_base) (void)hipFree(sv->pool_base);
  if (sv->hpin) (void)hipHostFree(sv->hpin);
  delete sv;
  return ZA_OK;
}

}  // extern "C"
