// Kernels of the WENO-ZA6 hot path for gfx950: sweeps, wave-speed
// reductions, RK3 stage updates.
#pragma once
#include "za_device.hpp"

namespace za {

// Global-memory view of a device pointer.  Every array a sweep reads or
// writes is device memory; the batched server kernels read their pointers
// from a table, where the compiler cannot see that and would otherwise use
// flat memory instructions (64-bit addresses in vector registers, and
// counted by the LDS wait counter as well, so that a wait for LDS data also
// waits for those loads).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

enum Sys { SYS_ADV = 0, SYS_EULER = 1, SYS_BURGERS = 2, SYS_BUCKLEY = 3 };
enum Mode {
  MODE_FLUX = 0,    // write the interface fluxes
  MODE_RHS = 1,     // write (x) / accumulate (y) L
  MODE_LX = 2,      // 2D stage, x-sweep: write ca Q^n + cb (Q + dt L_x) to workspace
  MODE_STAGE = 3    // last sweep of a stage: L (+ L_x) -> RK3 stage update
};

// Device control block: Lax-Friedrichs speeds of the current stage input,
// the step's dt, and the bookkeeping of a time integration.  Stays on the
// device so that whole RK3 steps run without host round trips.
struct DevCtl {
  double alpha[2][4];     // per direction, per characteristic field
  double smax[2];         // max(|u_n| + c) per direction
  double dt;              // dt of the step in progress
  double t;               // simulated time
  double t_final;         // clip target (infinity: no clipping)
  double dt_fixed;        // > 0: use this dt instead of the CFL rule
  double dt_min, dt_max;
  long long steps;        // completed steps
  long long max_steps;    // stop after this many (<= 0: no cap)
  long long bad_step;     // first step with a non-finite input, else -1
  int active;             // 1 while stepping
  int bad;                // non-finite / non-physical state seen
  int last;               // the step in progress lands on t_final
  int pad;
};

struct Geom {
  int nx, ny;
  int bc_x, bc_y;         // 0 periodic, 1 transmissive
  double inv_dx, inv_dy;
  double dx, dy;
};

struct Phys {
  double gm1;             // gamma - 1
  double gamma;
  double adv[2];          // advection velocity
  double cfl;
  int dt_rule;            // 0 CFL, 1 CFL h^2
  int lf_scalar;          // 1: one LF speed for every field
  int pp;                 // 1: positivity-preserving flux limiter in stages
};

// Ghost cells: periodic wrap or transmissive clamp (three per side).
__device__ __forceinline__ int bc_map(int j, int n, int bc) {
  if (bc == 0) {
    j = j < 0 ? j + n : j;
    j = j >= n ? j - n : j;
    // n >= 3 is required for a single wrap; smaller periodic grids use mod
    if (j < 0 || j >= n) { j %= n; if (j < 0) j += n; }
    return j;
  }
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// bc_map for a wavefront whose cells lie in [j0, j0 + span) with j0
// wave-uniform: away from the boundary (the usual case) a uniform branch
// skips the ghost rule and its integer arithmetic.
__device__ __forceinline__ int bc_map_span(int j, int j0, int span, int n, int bc) {
  if (j0 >= 0 && j0 + span <= n) return j;
  return bc_map(j, n, bc);
}

// ---------------------------------------------------------------------------
// Scalar flux functions and their derivatives (Section 2; Section 4.1).
// ---------------------------------------------------------------------------
template <int SYS, class T>
__device__ __forceinline__ T scalar_f(T u, T a) {
  if (SYS == SYS_ADV) return a * u;
  if (SYS == SYS_BURGERS) return T(0.5) * u * u;
  T s = u * u, w = T(1) - u;
  return s / (s + T(0.25) * (w * w));
}
template <int SYS>
__device__ __forceinline__ double scalar_df(double u, double a) {
  if (SYS == SYS_ADV) return a;
  if (SYS == SYS_BURGERS) return u;
  double D = u * u + 0.25 * (1 - u) * (1 - u);
  double Dp = 2 * u - 0.5 * (1 - u);
  return (2 * u * D - u * u * Dp) / (D * D);
}

// ---------------------------------------------------------------------------
// Wave speeds: per block maxima of |u_n - c|, |u_n|, |u_n + c| per direction
// (part[b][0..5] = ax0 ax1 ax3 ay0 ay1 ay3).  max(|u_n| + c) equals
// max(|u_n - c|, |u_n + c|) exactly (c > 0; both round the same sum), so it
// is not stored.  A non-finite or non-physical cell (rho <= 0, p <= 0) sets
// slot 0 to +infinity, which the final reduction reports.  Maxima are exact
// and order independent, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int NPART = 6;
constexpr int RED_BLOCKS_MAX = 1024;

__device__ __forceinline__ double wave_max(double a, double b) { return a > b ? a : b; }

// Velocities and sound speed of one Euler cell, each operation rounded once
// in the order u = m_x / rho, v = m_y / rho,
// p = (gamma-1) (E - (rho/2) (u^2 + v^2)), c^2 = gamma p / rho, c = sqrt(c^2),
// with correctly rounded division and square root and no contraction: the
// wave speeds, hence the Lax-Friedrichs speeds of eq:LF and the CFL step,
// are then exact functions of the state that any other correctly rounded
// evaluation in this order reproduces bit for bit.  Runs once per cell and
// stage.
__device__ __forceinline__ void euler_cell_speed(double rho, double mx, double my, double E, const Phys& ph,
                                                 double& u, double& v, double& p, double& c2) {
#pragma clang fp contract(off)
  u = mx / rho;
  v = my / rho;
  p = ph.gm1 * (E - 0.5 * rho * (u * u + v * v));
  c2 = ph.gamma * p / rho;
}

// acc = max(acc, |x|) for numbers acc, x (no NaN): one v_max_f64 with the
// absolute-value modifier, in place.  (fmax would make the compiler quiet
// possible signalling NaNs first, an extra instruction per operand and
// register copies around the loop that carries acc.)
__device__ __forceinline__ void max_abs_into(double& acc, double x) {
  asm("v_max_f64 %0, %0, |%1|" : "+v"(acc) : "v"(x));
}

template <int SYS, int M>
__device__ __forceinline__ void cell_speeds(const double (&Q)[M], const Phys& ph, double (&r)[NPART]) {
  if (SYS == SYS_EULER) {
    double u, v, p, c2;
    euler_cell_speed(Q[0], Q[1 % M], M == 4 ? Q[2 % M] : 0.0, Q[M - 1], ph, u, v, p, c2);
    // A NaN or infinite component makes p NaN, -inf or +inf (then c2 = +inf),
    // so these tests also reject every non-finite state; past them all
    // speeds are numbers and the maxima need no NaN care.  (A branch-free
    // form with a select on r[0] saves a few instructions but led the
    // compiler to reuse the registers of in-flight stores early, and the
    // waits for those stores cost 7 % of the y-sweep.)
    const bool ok = Q[0] > 0.0 && p > 0.0 && c2 > 0.0 && c2 < __builtin_huge_val();
    if (!ok) { r[0] = __builtin_huge_val(); return; }
    const double c = __builtin_sqrt(c2);
    max_abs_into(r[0], u - c);
    max_abs_into(r[1], u);
    max_abs_into(r[2], u + c);
    max_abs_into(r[3], v - c);
    max_abs_into(r[4], v);
    max_abs_into(r[5], v + c);

  } else if (SYS == SYS_BUCKLEY) {
    // non-convex flux: keep the data range (max u, max -u); the final
    // reduction takes max |f'| over it
    const double u = Q[0];
    if (!((u - u) == 0.0)) { r[0] = __builtin_huge_val(); return; }
    r[0] = wave_max(r[0], u);
    r[1] = wave_max(r[1], -u);
  } else {
    const double u = Q[0];
    if (!((u - u) == 0.0)) { r[0] = __builtin_huge_val(); return; }
    const double ax = fabs(scalar_df<SYS>(u, ph.adv[0]));
    const double ay = fabs(scalar_df<SYS>(u, ph.adv[1]));
    r[0] = wave_max(r[0], ax); r[2] = r[0];
    r[3] = wave_max(r[3], ay); r[5] = r[3];
  }
}

// Largest |f'(u)| of the Buckley-Leverett flux for u in [lo, hi]:
// f'(u) = u (1-u) / (2 D^2), D = u^2 + (1-u)^2/4, is extremal where
// 10 u^3 - 15 u^2 + 1 = 0 (one root in each of (-1/2, 0), (0, 1/2),
// (1, 3/2)); the maximum is at an end of the interval or at such a root
// inside it.  The roots are found by bisection to the last bit.
__device__ __forceinline__ double buckley_dfdu(double u) {
  const double w = 1.0 - u;
  const double D = fma(u, u, 0.25 * w * w);
  return 0.5 * u * w / (D * D);
}
__device__ inline double buckley_max_speed(double lo, double hi) {
  double best = fmax(fabs(buckley_dfdu(lo)), fabs(buckley_dfdu(hi)));
  const double b0[3] = {-0.5, 0.0, 1.0}, b1[3] = {0.0, 0.5, 1.5};
  for (int k = 0; k < 3; ++k) {
    double a = b0[k], c = b1[k];
    const bool neg_at_a = fma(fma(10.0, a, -15.0), a * a, 1.0) < 0.0;
    for (int it = 0; it < 200; ++it) {
      const double m = 0.5 * (a + c);
      if (!(m > a && m < c)) break;
      const bool neg = fma(fma(10.0, m, -15.0), m * m, 1.0) < 0.0;
      if (neg == neg_at_a) a = m; else c = m;
    }
    if (a > lo && a < hi) best = fmax(best, fabs(buckley_dfdu(a)));
  }
  return best;
}

// Index of the calling wavefront in its block, as a wave-uniform (scalar)
// value so that everything derived from it stays in scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Orders LDS traffic among the lanes of one wavefront.  The LDS unit serves
// a wavefront's requests in issue order, so it suffices to keep the compiler
// from moving memory operations across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide maxima of r into dst[0..NPART); every thread of the block calls.
__device__ __forceinline__ void block_max_store(double (&r)[NPART], double* __restrict__ dst) {
#pragma unroll
  for (int i = 0; i < NPART; ++i) {
    for (int off = 32; off > 0; off >>= 1) r[i] = wave_max(r[i], __shfl_xor(r[i], off, 64));
  }
  __shared__ double sm[8][NPART];
  const int lane = threadIdx.x & 63, wv = wave_id();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NPART; ++i) sm[wv][i] = r[i];
  }
  __syncthreads();
  if (threadIdx.x < NPART) {
    double v = sm[0][threadIdx.x];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = wave_max(v, sm[w][threadIdx.x]);
    gptr(dst)[threadIdx.x] = v;
  }
}

template <int SYS, int M>
__global__ __launch_bounds__(256) void k_wave_partial(const double* __restrict__ q, size_t ncell, Phys ph,
                                                      const DevCtl* ctl, int check_active,
                                                      double* __restrict__ part) {
  if (check_active && !ctl->active) return;
  double r[NPART];
#pragma unroll
  for (int i = 0; i < NPART; ++i) r[i] = -__builtin_huge_val();
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
    double Q[M];
#pragma unroll
    for (int c = 0; c < M; ++c) Q[c] = q[c * ncell + i];
    cell_speeds<SYS, M>(Q, ph, r);
  }
  block_max_store(r, part + (size_t)blockIdx.x * NPART);
}

// ---------------------------------------------------------------------------
// Records of one sweep direction (see za_device.hpp).  DIR 1 permutes the 2D
// Euler state into the sweep-normal frame (rho, rho v, rho u, E).
// ---------------------------------------------------------------------------
template <int SYS, int M>
struct NumFields { enum { value = (SYS == SYS_EULER) ? RecLayout<(M == 1 ? 4 : M)>::NF : 2 }; };

// Gather cell `off` (already boundary-mapped) of the line at `base` in the
// sweep-normal frame (DIR = 1 swaps the two momenta), and build a record at
// rec (field stride fs) from such a state.  Callers that stage several cells
// issue every load before the first record so the latencies overlap.
template <int SYS, int M, int DIR>
__device__ __forceinline__ void cell_load(const double* __restrict__ base, size_t cs, size_t off, double (&qd)[M]) {
  const auto* const b = gptr(base);
  if (SYS == SYS_EULER && M == 4 && DIR == 1) {
    qd[0] = b[off];
    qd[1 % M] = b[off + 2 * cs];
    qd[2 % M] = b[off + cs];
    qd[3 % M] = b[off + 3 * cs];
  } else if (SYS == SYS_EULER) {
#pragma unroll
    for (int c = 0; c < M; ++c) qd[c] = b[off + c * cs];
  } else {
    qd[0] = b[off];
  }
}

template <int SYS, int M, int DIR, class T>
__device__ __forceinline__ void cell_record(const double (&qd)[M], const Phys& ph, T* rec, int fs) {
  if (SYS == SYS_EULER) {
    euler_record<T, (M == 1 ? 4 : M)>(*reinterpret_cast<const double(*)[(M == 1 ? 4 : M)]>(qd), (T)ph.gm1, rec, fs);
  } else {
    const T u = (T)qd[0];
    rec[0] = u;
    rec[fs] = scalar_f<SYS, T>(u, (T)ph.adv[DIR]);
  }
}

// ---------------------------------------------------------------------------
// Positivity-preserving flux limiter (Euler, FP64 stages), after Hu, Adams
// and Shu (J. Comput. Phys. 242, 2013), cited by the paper for its shock
// diffraction test (Section 4.3).  A stage Q + dt L(Q) is a convex
// combination of 1D updates, and each direction's update of a cell is the
// mean of two half states, one per face: Q_i - 2 mu F_{i+1/2} and
// Q_{i+1} + 2 mu F_{i+1/2}, mu = dt S / s_dir (s_dir = max(|u_n| + c) of the
// direction, S = sum_d s_d / dx_d; 1D: mu = dt / dx).  With the first-order
// global LF flux both half states are positive for dt S <= 1/2; the face
// flux becomes F_LF + theta (F - F_LF) with the largest theta in [0, 1] (up
// to the bounds) keeping density and pressure of both half states >= 1e-13:
// density is linear in theta, pressure concave in the state, so the chord
// from the LF half state to the density-limited one bounds it from below.
// Works in the sweep-normal frame (density and pressure do not depend on the
// order of the momentum components).
// ---------------------------------------------------------------------------
constexpr double PP_EPS = 1e-13;

template <int M>
__device__ __forceinline__ double pp_pressure(const double (&U)[M], double gm1) {
  double k = U[1] * U[1];
  if (M == 4) k = fma(U[2 % M], U[2 % M], k);
  return gm1 * (U[M - 1] - 0.5 * k / U[0]);
}

// theta keeping A + theta B admissible (A: a half state of the LF flux)
template <int M>
__device__ __forceinline__ double pp_theta(const double (&A)[M], const double (&B)[M], double gm1) {
  const double rA = A[0];
  const double pA = rA > 0.0 ? pp_pressure<M>(A, gm1) : -1.0;
  if (!(rA >= PP_EPS) || !(pA >= PP_EPS)) return 0.0;
  double th = 1.0;
  const double r1 = rA + B[0];
  if (r1 < PP_EPS) th = (rA - PP_EPS) / (rA - r1);
  double U1[M];
#pragma unroll
  for (int c = 0; c < M; ++c) U1[c] = fma(th, B[c], A[c]);
  const double p1 = pp_pressure<M>(U1, gm1);
  if (p1 < PP_EPS) th = th * (pA - PP_EPS) / (pA - p1);
  return th;
}

// Limit the sweep-frame flux F of the face between the records at oL, oR.
template <int M>
__device__ void pp_limit_face(const double* __restrict__ rec, int fs, int oL, int oR, double gm1, double s,
                              double mu, double (&F)[M]) {
  typedef RecLayout<M> Lo;
  double QL[M], QR[M], FL[M], FR[M];
  QL[0] = rec[Lo::Q0 * fs + oL];  QR[0] = rec[Lo::Q0 * fs + oR];
  QL[1] = rec[Lo::Q1 * fs + oL];  QR[1] = rec[Lo::Q1 * fs + oR];
  QL[M - 1] = rec[Lo::E * fs + oL];  QR[M - 1] = rec[Lo::E * fs + oR];
  FL[0] = QL[1];  FR[0] = QR[1];
  FL[1] = rec[Lo::F1 * fs + oL];  FR[1] = rec[Lo::F1 * fs + oR];
  FL[M - 1] = rec[Lo::F3 * fs + oL];  FR[M - 1] = rec[Lo::F3 * fs + oR];
  if (M == 4) {
    QL[2 % M] = rec[(M == 4 ? Lo::Q2 : 0) * fs + oL];  QR[2 % M] = rec[(M == 4 ? Lo::Q2 : 0) * fs + oR];
    FL[2 % M] = rec[(M == 4 ? Lo::F2 : 0) * fs + oL];  FR[2 % M] = rec[(M == 4 ? Lo::F2 : 0) * fs + oR];
  }
  double Flf[M], AL[M], BL[M], AR[M], BR[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    Flf[c] = 0.5 * (FL[c] + FR[c] - s * (QR[c] - QL[c]));
    const double d = 2.0 * mu * (F[c] - Flf[c]);
    AL[c] = QL[c] - 2.0 * mu * Flf[c];
    BL[c] = -d;
    AR[c] = QR[c] + 2.0 * mu * Flf[c];
    BR[c] = d;
  }
  const double th = fmin(pp_theta<M>(AL, BL, gm1), pp_theta<M>(AR, BR, gm1));
  if (th < 1.0) {
#pragma unroll
    for (int c = 0; c < M; ++c) F[c] = fma(th, F[c] - Flf[c], Flf[c]);
  }
}

// Constants of one sweep launch, read from the control block before the
// sweep writes anything (so they load once, into scalar registers): the LF
// speeds of the sweep direction, dt, the direction's max(|u_n| + c) and the
// limiter step size mu = dt S / s_DIR (0: no limiting).
struct SweepConst {
  double al[4];
  double dt, smax, mu;
};

template <int DIR>
__device__ __forceinline__ SweepConst sweep_const(const DevCtl* ctl_, const Geom& g, bool pp, bool two_d) {
  const auto* const ctl = gptr(ctl_);
  SweepConst k;
#pragma unroll
  for (int s = 0; s < 4; ++s) k.al[s] = ctl->alpha[DIR][s];
  k.dt = ctl->dt;
  k.smax = ctl->smax[DIR];
  k.mu = 0.0;
  if (pp) {
    const double sx = ctl->smax[0], sy = two_d ? ctl->smax[1] : 0.0;
    const double S = fma(sx, g.inv_dx, two_d ? sy * g.inv_dy : 0.0);
    const double sd = DIR == 0 ? sx : sy;
    k.mu = sd > 0.0 ? k.dt * S / sd : 0.0;
  }
  return k;
}

// Interface flux from the records of its six-point stencil; the result is
// returned in the state's own component order.
template <int SYS, int M, int DIR, class T, int WV, int R = 3>
__device__ __forceinline__ void stencil_flux(const T* __restrict__ rec, int fs, const int (&off)[2 * R],
                                             const Phys& ph, const SweepConst& sk, const WeightCfg<T>& cfg,
                                             T (&Fh)[M]) {
  if (SYS == SYS_EULER) {
    constexpr int MM = (M == 1 ? 4 : M);
    T al[MM];
    if (MM == 4) {
      al[0] = (T)sk.al[0]; al[1] = (T)sk.al[1];
      al[2 % MM] = (T)sk.al[2]; al[3 % MM] = (T)sk.al[3];
    } else {
      al[0] = (T)sk.al[0]; al[1] = (T)sk.al[1]; al[MM - 1] = (T)sk.al[3];
    }
    T F[MM];
    euler_flux<T, MM, WV, R>(rec, fs, off, (T)ph.gm1, al, cfg, F);
    if constexpr (sizeof(T) == sizeof(double)) {
      if (sk.mu > 0.0) {
        double Fd[MM];
#pragma unroll
        for (int c = 0; c < MM; ++c) Fd[c] = (double)F[c];
        pp_limit_face<MM>(reinterpret_cast<const double*>(rec), fs, off[R - 1], off[R], ph.gm1, sk.smax, sk.mu, Fd);
#pragma unroll
        for (int c = 0; c < MM; ++c) F[c] = (T)Fd[c];
      }
    }
    if (MM == 4 && DIR == 1) {
      Fh[0] = F[0]; Fh[1 % M] = F[2 % MM]; Fh[2 % M] = F[1]; Fh[3 % M] = F[3 % MM];
    } else {
#pragma unroll
      for (int c = 0; c < M; ++c) Fh[c] = F[c];
    }
  } else {
    T w[2 * R], g[2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
      w[j] = rec[off[j]];
      g[j] = rec[fs + off[j]];
    }
    Fh[0] = split_pair<T, WV, R>(w, g, (T)sk.al[0], cfg);
  }
}

struct SweepArgs {
  const double* q;       // sweep input Q^(s)
  const double* qn;      // Q^n (stage update)
  const double* lx;      // 2D: L_x (rhs) or the x-sweep's partial stage update
  double* out;           // L, L_x, Q^(s+1) or fluxes
  DevCtl* ctl;
  Geom g;
  Phys ph;
  double ca, cb;         // stage: out = ca*qn + cb*(q + dt*L)
  int check_active;      // stepping: skip when the integration is inactive
  int ytile;             // y-sweep: at most this many rows per block (band)
  double* part;          // MODE_STAGE: per-block wave-speed maxima of the new state
  int xl_chunks;         // looped x-sweep: 64-interface chunks per row segment
};

template <class T>
struct CfgArg { WeightCfg<T> w; };

// ---------------------------------------------------------------------------
// x-sweep: one wavefront per line segment of 64 interfaces / 63 cells.  The
// wavefront first builds the records of its 63 + 2R cells (the cells and the
// stencil halo, coalesced loads; R = 3: 69) in LDS; each lane then computes
// one interface flux from 2R consecutive records, and the fluxes meet in LDS
// again for the conservative difference.  Used for the 2D x-direction and
// for 1D problems.
// ---------------------------------------------------------------------------
constexpr int XS_CELLS = 63;
#ifndef ZA_XS_WAVES
#define ZA_XS_WAVES 4   // minimum resident wavefronts per SIMD requested from the compiler
#endif
#ifndef ZA_YS_WAVES
#define ZA_YS_WAVES 3
#endif
// record slots per field and wavefront: the 63 cells and a 2R-cell halo
__host__ __device__ constexpr int xs_rec(int R) { return (XS_CELLS + 2 * R + 7) / 8 * 8; }

template <int SYS, int M, class T, int MODE, int WV, int R = 3, int PP = 0>
__device__ __forceinline__ void sweep_x_body(const SweepArgs& a, const CfgArg<T>& cfg, int bid) {
  constexpr int XS_REC = xs_rec(R);
  if (a.check_active && !gptr(a.ctl)->active) return;
  const SweepConst sk = sweep_const<0>(a.ctl, a.g, PP && SYS == SYS_EULER && (MODE == MODE_LX || MODE == MODE_STAGE),
                                       MODE == MODE_LX);
  constexpr int NF = NumFields<SYS, M>::value;
  __shared__ T xr[4][NF * XS_REC];
  __shared__ double fl[4][M][64];
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int nx = a.g.nx, ny = a.g.ny;
  const int nseg = (nx + XS_CELLS - 1) / XS_CELLS;
  const long long wid = (long long)bid * 4 + wv;
  const int line = (int)(wid / nseg), seg = (int)(wid % nseg);
  const bool live = line < ny;
  const int c0 = seg * XS_CELLS;
  const int k = c0 + lane;
  const size_t cs = (size_t)nx * ny;
  const size_t row = (size_t)line * nx;
  if (live) {
    constexpr int NX = (XS_CELLS + 2 * R + 63) / 64;   // record passes
    double qx[NX][M];
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int idx = lane + 64 * t;
      if (idx < XS_CELLS + 2 * R)
        cell_load<SYS, M, 0>(a.q + row, cs, (size_t)bc_map_span(c0 - R + idx, c0 - R + 64 * t, 64, nx, a.g.bc_x),
                             qx[t]);
    }
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int idx = lane + 64 * t;
      if (idx < XS_CELLS + 2 * R) cell_record<SYS, M, 0, T>(qx[t], a.ph, &xr[wv][idx], XS_REC);
    }
  }
  wave_sync();   // the records and fluxes of a wavefront are its own
  if (live && k <= nx) {
    T F[M];
    int off[2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) off[j] = lane + j;
    stencil_flux<SYS, M, 0, T, WV, R>(&xr[wv][0], XS_REC, off, a.ph, sk, cfg.w, F);
    if (MODE == MODE_FLUX) {
      if (lane < XS_CELLS || k == nx) {
#pragma unroll
        for (int c = 0; c < M; ++c) gptr(a.out)[(size_t)c * ny * (nx + 1) + (size_t)line * (nx + 1) + k] = (double)F[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < M; ++c) fl[wv][c][lane] = (double)F[c];
    }
  }
  if (MODE == MODE_FLUX) return;
  wave_sync();
  const int i = c0 + lane;
  double rs[NPART];
#pragma unroll
  for (int t = 0; t < NPART; ++t) rs[t] = -__builtin_huge_val();
  if (live && lane < XS_CELLS && i < nx) {
    const size_t idx = row + i;
    if (MODE == MODE_LX) {
      // partial stage ca Q^n + cb (Q + dt L_x); FP64 records hold Q exactly
      double qc[M], qb[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        if (sizeof(T) == sizeof(double) && SYS == SYS_EULER) {
          typedef RecLayout<(M == 1 ? 4 : M)> Lo;
          const int f = c == 0 ? (int)Lo::Q0 : (c == M - 1 ? (int)Lo::E : (c == 1 ? (int)Lo::Q1 : (int)Lo::Q2));
          qc[c] = (double)xr[wv][f * XS_REC + lane + R];
        } else if (sizeof(T) == sizeof(double)) {
          qc[c] = (double)xr[wv][lane + R];
        } else {
          qc[c] = gptr(a.q)[c * cs + idx];
        }
      }
      if (a.ca != 0.0) {
#pragma unroll
        for (int c = 0; c < M; ++c) qb[c] = gptr(a.qn)[c * cs + idx];
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) qb[c] = 0.0;
      }
      // ca Q^n + cb Q - cb dt (F_{i+1/2} - F_{i-1/2}) / dx, the same
      // operations as the looped sweep
      const double kx = -(a.cb * sk.dt) * a.g.inv_dx;
#pragma unroll
      for (int c = 0; c < M; ++c)
        gptr(a.out)[c * cs + idx] = fma(a.ca, qb[c], fma(kx, fl[wv][c][lane + 1] - fl[wv][c][lane], a.cb * qc[c]));
    } else {
      double qnew[M], q0[M], qs[M];
      if (MODE == MODE_STAGE) {   // loads first (see the y-sweep epilogue)
#pragma unroll
        for (int c = 0; c < M; ++c) { q0[c] = gptr(a.qn)[c * cs + idx]; qs[c] = gptr(a.q)[c * cs + idx]; }
      }
      const double kx = -(a.cb * sk.dt) * a.g.inv_dx;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const size_t o = c * cs + idx;
        if (MODE == MODE_RHS) {
          gptr(a.out)[o] = -(fl[wv][c][lane + 1] - fl[wv][c][lane]) * a.g.inv_dx;
        } else {  // MODE_STAGE (1D)
          qnew[c] = fma(a.ca, q0[c], fma(kx, fl[wv][c][lane + 1] - fl[wv][c][lane], a.cb * qs[c]));
          gptr(a.out)[o] = qnew[c];
        }
      }
      if (MODE == MODE_STAGE) cell_speeds<SYS, M>(qnew, a.ph, rs);
    }
  }
  if (MODE == MODE_STAGE && a.part) block_max_store(rs, a.part + (size_t)bid * NPART);
}

// ---------------------------------------------------------------------------
// Looped x-sweep of a stage (FP64 records): one wavefront per row segment of
// 64 nc - 1 cells, walked in nc chunks of 64 interfaces.  Lane l of chunk j
// computes interface I0 + l (I0 = s0 + 64 j) from a 128-cell LDS ring of
// records; each chunk first adds the next 64 cells to the ring (their state
// was loaded while the previous chunk computed its fluxes) and then updates
// cell I0 - 1 + l, whose left flux the previous chunk's lane 63 left in a
// carry slot.  Every record is built once per segment, and neighbouring
// segments share one interface, so a row of 2048 cells takes the same 33 flux
// passes as the one-shot sweep with half its record passes.
//   MODE_LX (2D): the partial stage ca Q^n + cb (Q + dt L_x).
//   MODE_STAGE (1D): the whole RK3 stage, and the wave-speed maxima of the new
//   states, one row of a.part per wavefront (row = global wavefront index;
//   the ny * nseg live wavefronts fill rows 0 .. ny * nseg - 1).
// ---------------------------------------------------------------------------
constexpr int XL_RING = 128;

// live wavefronts of the looped sweep: ny rows of segments of 64 nc - 1 cells
__host__ __device__ constexpr long long xl_waves(int nx, int ny, int nc) {
  return (long long)ny * ((nx + 64LL * nc - 2) / (64LL * nc - 1));
}

__device__ __forceinline__ int xl_slot(int k) { return k & (XL_RING - 1); }

// Write-only target of the looped sweep's lanes that have no cell to store
// (component c of lane l at [64 c + l]); nothing reads it.
static __device__ double xl_sink[4 * 64];

template <int SYS, int M>
__device__ __forceinline__ void xl_load(const double* __restrict__ row, size_t cs, int j, double (&qp)[M]) {
#pragma unroll
  for (int c = 0; c < M; ++c) qp[c] = gptr(row)[(size_t)j + c * cs];
}

template <int SYS, int M>
__device__ __forceinline__ void xl_record(const double (&qp)[M], const Phys& ph, double* rec) {
  if (SYS == SYS_EULER) {
    euler_record<double, (M == 1 ? 4 : M)>(*reinterpret_cast<const double(*)[(M == 1 ? 4 : M)]>(qp), ph.gm1, rec,
                                           XL_RING);
  } else {
    rec[0] = qp[0];
    rec[XL_RING] = scalar_f<SYS, double>(qp[0], ph.adv[0]);
  }
}

// The maxima of a wavefront's lanes to dst[0 .. NPART-1] (lane 0 stores).
// cell_speeds leaves numbers or +inf, never NaN, so fmax is the exact max.
__device__ __forceinline__ void wave_max_store(double (&r)[NPART], double* __restrict__ dst) {
#pragma unroll
  for (int i = 0; i < NPART; ++i) {
    for (int off = 32; off > 0; off >>= 1) r[i] = fmax(r[i], __shfl_xor(r[i], off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NPART; ++i) gptr(dst)[i] = r[i];
  }
}

template <int SYS, int M, int WV, int MODE = MODE_LX>
__device__ __forceinline__ void sweep_xl_body(const SweepArgs& a, const CfgArg<double>& cfg, int bid) {
  static_assert(MODE == MODE_LX || MODE == MODE_STAGE, "the looped sweep writes stage states");
  constexpr int R = 3;
  if (a.check_active && !gptr(a.ctl)->active) return;
  const SweepConst sk = sweep_const<0>(a.ctl, a.g, false, MODE == MODE_LX);
  constexpr int NF = NumFields<SYS, M>::value;
  __shared__ double xr[4][NF * XL_RING];
  __shared__ double fl[4][M][66];   // [l + 1]: flux of lane l; [65]: carry from the previous chunk
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int nx = a.g.nx, ny = a.g.ny;
  const int nc = a.xl_chunks;
  if (nc < 1) return;   // launched only with nc >= 1; never index with a negative segment
  const int seg_cells = 64 * nc - 1;
  const int nseg = (nx + seg_cells - 1) / seg_cells;
  const int wid = bid * 4 + wv;
  const int line = wid / nseg, seg = wid - line * nseg;   // wave-uniform
  if (line >= ny) return;   // the wavefronts of a block never wait for each other
  const int s0 = seg * seg_cells;
  const int nch = min(nc, (nx - s0) / 64 + 1);   // chunks holding interfaces <= nx
  const size_t cs = (size_t)nx * ny;
  const double* const rowq = a.q + (size_t)line * nx;
  double* const ring = &xr[wv][0];
  double(*const fw)[66] = fl[wv];
  const int bcx = a.g.bc_x;
  // ca Q^n + cb Q - cb dt (F_{i+1/2} - F_{i-1/2}) / dx
  const double kx = -(a.cb * sk.dt) * a.g.inv_dx;
  // ring slot of cell k is (k - s0 + R) mod 128; cells s0 - R .. s0 - R + 63 first
  double rs[NPART];
#pragma unroll
  for (int t = 0; t < NPART; ++t) rs[t] = -__builtin_huge_val();
  double qp[M];
  {
    double q0[M];   // both loads in flight before the first records
    xl_load<SYS, M>(rowq, cs, bc_map(s0 - R + lane, nx, bcx), q0);
    xl_load<SYS, M>(rowq, cs, bc_map(s0 - R + 64 + lane, nx, bcx), qp);
    xl_record<SYS, M>(q0, a.ph, ring + lane);
    xl_record<SYS, M>(qp, a.ph, ring + xl_slot(64 + lane));
  }
  for (int j = 0; j < nch; ++j) {
    const int I0 = s0 + 64 * j;
    wave_sync();   // the records of cells I0 - R .. I0 + 124 - R are in the ring
    if (j + 1 < nch) xl_load<SYS, M>(rowq, cs, bc_map_span(I0 + 128 - R + lane, I0 + 128 - R, 64, nx, bcx), qp);
    // the cell this lane completes, and its Q^n (fetched before the fluxes)
    const int i = I0 - 1 + lane;
    const bool upd = (j > 0 || lane > 0) && i < nx;
    double qb[M];
#pragma unroll
    for (int c = 0; c < M; ++c) qb[c] = 0.0;
    if (upd && a.ca != 0.0) {
#pragma unroll
      for (int c = 0; c < M; ++c) qb[c] = gptr(a.qn)[c * cs + (size_t)line * nx + i];
    }
    const int I = I0 + lane;
    double F[M];
    if (I <= nx) {
      int off[2 * R];
#pragma unroll
      for (int jj = 0; jj < 2 * R; ++jj) off[jj] = xl_slot(64 * j + lane + jj);
      stencil_flux<SYS, M, 0, double, WV, R>(ring, XL_RING, off, a.ph, sk, cfg.w, F);
#pragma unroll
      for (int c = 0; c < M; ++c) fw[c][lane + 1] = F[c];
    }
    wave_sync();
    {
      // Every lane stores, those without a cell of their own (the first
      // lane of the first chunk, whose cell the previous segment completes,
      // and lanes past the row's end) into xl_sink: with no branch around
      // the stores, each chunk issues the same memory operations, and the
      // wait for the next chunk's cells below never waits for these stores.
      const int si = xl_slot(64 * j + lane - 1 + R);
      auto* d = upd ? gptr(a.out) + (size_t)line * nx + i : gptr(xl_sink) + lane;
      const size_t dstride = upd ? cs : 64;
      double qnew[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        double qc;
        if (SYS == SYS_EULER) {
          typedef RecLayout<(M == 1 ? 4 : M)> Lo;
          const int f = c == 0 ? (int)Lo::Q0 : (c == M - 1 ? (int)Lo::E : (c == 1 ? (int)Lo::Q1 : (int)Lo::Q2));
          qc = ring[f * XL_RING + si];
        } else {
          qc = ring[si];
        }
        const double Fm = lane == 0 ? fw[c][65] : fw[c][lane];
        qnew[c] = fma(a.ca, qb[c], fma(kx, fw[c][lane + 1] - Fm, a.cb * qc));
        *d = qnew[c];
        d += dstride;
      }
      if (MODE == MODE_STAGE && upd) cell_speeds<SYS, M>(qnew, a.ph, rs);
    }
    wave_sync();
    if (lane == 63 && I <= nx) {
#pragma unroll
      for (int c = 0; c < M; ++c) fw[c][65] = fw[c][64];
    }
    // the 64 cells the next chunk adds, I0 + 128 - R + lane, over the slots
    // of cells I0 - R + lane, which this chunk was the last to read
    if (j + 1 < nch) xl_record<SYS, M>(qp, a.ph, ring + xl_slot(64 * j + 128 + lane));
  }
  if (MODE == MODE_STAGE && a.part) wave_max_store(rs, a.part + (size_t)wid * NPART);
}

template <int SYS, int M, int WV, int MODE = MODE_LX>
__global__ __launch_bounds__(256, 3) void k_sweep_xl(SweepArgs a, CfgArg<double> cfg) {
  sweep_xl_body<SYS, M, WV, MODE>(a, cfg, blockIdx.x);
}

// ---------------------------------------------------------------------------
// y-sweep (2D): a block of four wavefronts owns 64 columns and a band of at
// most a.ytile rows (chosen on the host so that one round of resident blocks
// covers the grid).  Each wavefront marches down its own YS_COLS columns,
// YS_ROWS interface rows per step (lane = YS_COLS * row + column, so every
// global access covers whole 128-byte row segments).  The records of the
// YS_ROWS + 5 cell rows one step's stencils touch sit in a private LDS
// ring; a step loads the next YS_ROWS cell rows, computes its fluxes, writes
// the conservative differences (in MODE_STAGE added to the x-sweep's partial
// update, which completes the RK3 stage) and only then turns the loaded rows
// into records in the slots of the rows no later stencil needs.  Wavefronts
// never wait for each other.
// ---------------------------------------------------------------------------
constexpr int YS_TILE_MIN = 16;
constexpr int YS_COLS = 16;
constexpr int YS_ROWS = 64 / YS_COLS;
constexpr int YS_FSLOT = YS_ROWS + 1;
// record rows of one step's stencils (R = 3: 9)
__host__ __device__ constexpr int ys_ring(int R) { return YS_ROWS + 2 * R - 1; }

// Issue priority of a wavefront that has done step st of nst: it falls as the
// wavefront advances, so each SIMD favours the wavefronts that are behind and
// all of them finish at about the same time.  (Among equal priorities the
// oldest wavefront issues first, which would finish the first-dispatched
// tiles early and leave the last ones running alone at the end.)
__device__ __forceinline__ void progress_prio(int st, int nst) {
  const int q = (4 * st) / nst;
  if (q == 0) __builtin_amdgcn_s_setprio(3);
  else if (q == 1) __builtin_amdgcn_s_setprio(2);
  else if (q == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// One wavefront's tile: columns x0 .. x0+YS_COLS-1, cell rows [y0, ylast)
// (interfaces y0 .. ylast).  MODE_STAGE folds the wave speeds of the new
// states into rs.
template <int SYS, int M, class T, int MODE, int WV, int R = 3, int PP = 0>
__device__ __forceinline__ void sweep_y_tile(const SweepArgs& a, const CfgArg<T>& cfg, const SweepConst& sk, int x0,
                                             int y0, int ylast, double (&rs)[NPART]) {
  constexpr int YS_RING = ys_ring(R);
  constexpr int NF = NumFields<SYS, M>::value;
  constexpr int RS = NF * YS_COLS + 32 / (int)sizeof(T);   // ring row stride, padded by 32 bytes
  __shared__ T ring[4][YS_RING * RS];
  __shared__ double fb[4][YS_FSLOT][M][YS_COLS];
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int cl = lane % YS_COLS, g = lane / YS_COLS;
  const int nx = a.g.nx, ny = a.g.ny;
  const int x = x0 + cl;
  const bool xin = x < nx;
  const int kend = ylast;                    // interfaces y0 .. kend
  const size_t cs = (size_t)nx * ny;
  const int xc = xin ? x : 0;   // column offset of this lane's loads
  T* const rw = &ring[wv][cl];
  double(*const fw)[M][YS_COLS] = fb[wv];
  // Ring slot of cell row r is (r - y0 + R) mod YS_RING; flux slot of
  // interface k is (k - y0 + 1) mod YS_FSLOT.  Both advance by YS_ROWS per
  // step, so each lane carries them (scaled) instead of dividing.
  // rows y0-R .. y0+YS_ROWS+R-2 for the first step
  {
    constexpr int NPRO = (YS_RING + YS_ROWS - 1) / YS_ROWS;
    double qr[NPRO][M];
#pragma unroll
    for (int t = 0; t < NPRO; ++t) {
      const int i = g + YS_ROWS * t;
      if (xin && i < YS_RING)
        cell_load<SYS, M, 1>(a.q, cs, (size_t)bc_map(y0 - R + i, ny, a.g.bc_y) * nx + xc, qr[t]);
    }
#pragma unroll
    for (int t = 0; t < NPRO; ++t) {
      const int i = g + YS_ROWS * t;
      if (xin && i < YS_RING) cell_record<SYS, M, 1, T>(qr[t], a.ph, rw + i * RS, YS_COLS);
    }
  }
  wave_sync();
  // sb: slot of row k - R (the stencil's first row, and the slot that row
  // k0 + YS_ROWS + R - 1 + g takes at the end of the step), times RS;
  // fk: flux slot of interface k, fkm of k - 1
  int sb = g * RS;
  int fk = g + 1, fkm = g;
  constexpr int RING_RS = YS_RING * RS;
  const double ky = -(a.cb * sk.dt) * a.g.inv_dy;
  const int nst = (kend - y0) / YS_ROWS + 1;
  for (int st = 0; st < nst; ++st) {
    progress_prio(st, nst);
    const int k0 = y0 + YS_ROWS * st;
    const int k = k0 + g;
    const bool act = k <= kend && xin;
    // the cell row this lane adds for the next step's stencils
    const int rn = k0 + YS_ROWS + R - 1 + g;
    const bool need = rn <= kend + R - 1 && xin;
    double qp[M];
    if (need) {
      const size_t off = (size_t)bc_map_span(rn, k0 + YS_ROWS + R - 1, YS_ROWS, ny, a.g.bc_y) * nx;
#pragma unroll
      for (int c = 0; c < M; ++c) qp[c] = gptr(a.q)[off + xc + c * cs];
    }
    const int r = k - 1;   // cell row finished by this lane
    const bool upd = MODE != MODE_FLUX && act && r >= y0 && r < ylast;
    const size_t idx = (size_t)r * nx + x;
    // the x-sweep's part of this row's update, fetched before the fluxes
    double lx[M];
    if (upd) {
#pragma unroll
      for (int c = 0; c < M; ++c) lx[c] = gptr(a.lx)[c * cs + idx];
    }
    if (act) {
      T F[M];
      int off[2 * R];
      off[0] = sb;
#pragma unroll
      for (int j = 1; j < 2 * R; ++j) {
        const unsigned t = (unsigned)(sb + j * RS);
        off[j] = (int)min(t, t - (unsigned)RING_RS);   // t - RING_RS wraps above t when t < RING_RS
      }
      stencil_flux<SYS, M, 1, T, WV, R>(rw, YS_COLS, off, a.ph, sk, cfg.w, F);
#pragma unroll
      for (int c = 0; c < M; ++c) fw[fk][c][cl] = (double)F[c];
      if (MODE == MODE_FLUX && (k < kend || k == ny)) {
#pragma unroll
        for (int c = 0; c < M; ++c) gptr(a.out)[(size_t)c * (ny + 1) * nx + (size_t)k * nx + x] = (double)F[c];
      }
    }
    wave_sync();
    if (need) {
      // row rn takes the slot of row rn - YS_RING = k0 - R + g, which only
      // this step's stencils (above the synchronisation) read.  Built
      // before the update's stores: waiting for the loaded row then never
      // waits for stores.
      T* rec = rw + sb;
      if (SYS == SYS_EULER) {
        double qd[M];
        if (M == 4) { qd[0] = qp[0]; qd[1] = qp[2 % M]; qd[2 % M] = qp[1]; qd[3 % M] = qp[3 % M]; }
        else {
#pragma unroll
          for (int c = 0; c < M; ++c) qd[c] = qp[c];
        }
        euler_record<T, (M == 1 ? 4 : M)>(*reinterpret_cast<const double(*)[(M == 1 ? 4 : M)]>(qd), (T)a.ph.gm1, rec, YS_COLS);
      } else {
        const T u = (T)qp[0];
        rec[0] = u;
        rec[YS_COLS] = scalar_f<SYS, T>(u, (T)a.ph.adv[1]);
      }
    }
    if (upd) {
      double qnew[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double dF = fw[fk][c][cl] - fw[fkm][c][cl];
        const size_t o = c * cs + idx;
        if (MODE == MODE_RHS) {
          gptr(a.out)[o] = lx[c] - dF * a.g.inv_dy;
        } else {  // MODE_STAGE: the x-sweep left ca Q^n + cb Q - cb dt dF_x / dx
          qnew[c] = fma(ky, dF, lx[c]);
          gptr(a.out)[o] = qnew[c];
        }
      }
      if (MODE == MODE_STAGE) cell_speeds<SYS, M>(qnew, a.ph, rs);
    }
    wave_sync();
    // advance by YS_ROWS rows (YS_ROWS < YS_RING, YS_ROWS < YS_FSLOT)
    sb += YS_ROWS * RS;
    sb = (int)min((unsigned)sb, (unsigned)(sb - RING_RS));
    fkm = fk + YS_ROWS - 1;
    fkm = fkm >= YS_FSLOT ? fkm - YS_FSLOT : fkm;
    fk = fkm + 1 == YS_FSLOT ? 0 : fkm + 1;
  }
}

// Block (bx, by) owns 64 columns, one YS_COLS-column tile per wavefront, and
// band by of the ceil(ny / ytile) bands of (near) equal height.
template <int SYS, int M, class T, int MODE, int WV, int R = 3, int PP = 0>
__device__ __forceinline__ void sweep_y_body(const SweepArgs& a, const CfgArg<T>& cfg, int bx, int by, int gx) {
  if (a.check_active && !gptr(a.ctl)->active) return;
  const SweepConst sk = sweep_const<1>(a.ctl, a.g, PP && SYS == SYS_EULER && MODE == MODE_STAGE, true);
  double rs[NPART];
#pragma unroll
  for (int t = 0; t < NPART; ++t) rs[t] = -__builtin_huge_val();
  const int ny = a.g.ny;
  const int nb = (ny + a.ytile - 1) / a.ytile;
  const int y0 = (int)((long long)by * ny / nb), ylast = (int)((long long)(by + 1) * ny / nb);
  sweep_y_tile<SYS, M, T, MODE, WV, R, PP>(a, cfg, sk, bx * 64 + wave_id() * YS_COLS, y0, ylast, rs);
  if (MODE == MODE_STAGE && a.part)
    block_max_store(rs, a.part + ((size_t)by * gx + bx) * NPART);
}

// The fast variants (Z weights, p = 1, a stage or RHS mode) carry an
// occupancy target; the others (general weights, flux output for checks)
// let the compiler use as many registers as it likes.
template <int SYS, int M, class T, int MODE, int WV>
__global__ __launch_bounds__(256, ZA_XS_WAVES) void k_sweep_x(SweepArgs a, CfgArg<T> cfg) {
  sweep_x_body<SYS, M, T, MODE, WV>(a, cfg, blockIdx.x);
}
template <int SYS, int M, class T, int MODE, int WV, int R = 3>
__global__ __launch_bounds__(256) void k_sweep_x_any(SweepArgs a, CfgArg<T> cfg) {
  sweep_x_body<SYS, M, T, MODE, WV, R>(a, cfg, blockIdx.x);
}
template <int SYS, int M, class T, int MODE, int WV>
__global__ __launch_bounds__(256, ZA_YS_WAVES) void k_sweep_y(SweepArgs a, CfgArg<T> cfg) {
  sweep_y_body<SYS, M, T, MODE, WV>(a, cfg, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int SYS, int M, class T, int MODE, int WV, int R = 3>
__global__ __launch_bounds__(256) void k_sweep_y_any(SweepArgs a, CfgArg<T> cfg) {
  sweep_y_body<SYS, M, T, MODE, WV, R>(a, cfg, blockIdx.x, blockIdx.y, gridDim.x);
}
// Stages with the positivity-preserving limiter (Euler, FP64, r = 3).
template <int M, int MODE, int WV>
__global__ __launch_bounds__(256) void k_sweep_x_pp(SweepArgs a, CfgArg<double> cfg) {
  sweep_x_body<SYS_EULER, M, double, MODE, WV, 3, 1>(a, cfg, blockIdx.x);
}
template <int MODE, int WV>
__global__ __launch_bounds__(256) void k_sweep_y_pp(SweepArgs a, CfgArg<double> cfg) {
  sweep_y_body<SYS_EULER, 4, double, MODE, WV, 3, 1>(a, cfg, blockIdx.x, blockIdx.y, gridDim.x);
}
// Other orders with Z weights: an occupancy target per stencil width.
template <int SYS, int M, class T, int MODE, int WV, int R, int WAVES>
__global__ __launch_bounds__(256, WAVES) void k_sweep_x_r(SweepArgs a, CfgArg<T> cfg) {
  sweep_x_body<SYS, M, T, MODE, WV, R>(a, cfg, blockIdx.x);
}
template <int SYS, int M, class T, int MODE, int WV, int R, int WAVES>
__global__ __launch_bounds__(256, WAVES) void k_sweep_y_r(SweepArgs a, CfgArg<T> cfg) {
  sweep_y_body<SYS, M, T, MODE, WV, R>(a, cfg, blockIdx.x, blockIdx.y, gridDim.x);
}


__device__ __forceinline__ void step_end_body(DevCtl* ctl) {
  if (threadIdx.x != 0 || !ctl->active) return;
  const double dt = ctl->dt;
  ctl->t = ctl->last ? ctl->t_final : ctl->t + dt;
  ctl->steps += 1;
  ctl->dt_min = fmin(ctl->dt_min, dt);
  ctl->dt_max = fmax(ctl->dt_max, dt);
  if (ctl->last) ctl->active = 0;
  if (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps) ctl->active = 0;
}

// FIN_END_STAGE0: the previous step's end (step_end_body), then FIN_STAGE0,
// in one launch.
enum FinalKind { FIN_RHS = 0, FIN_STAGE0 = 1, FIN_STAGEK = 2, FIN_END_STAGE0 = 3 };

__device__ __forceinline__ void wave_final_body(const double* __restrict__ part, int nblk, DevCtl* ctl,
                                                const Geom& g, const Phys& ph, int dim, int kind, int sys) {
  // every thread of the block (one or more wavefronts) folds a strided share
  // of the per-block maxima; the maxima are exact whatever the order
  double r[NPART];
#pragma unroll
  for (int i = 0; i < NPART; ++i) r[i] = -__builtin_huge_val();
#pragma unroll 2
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int i = 0; i < NPART; ++i) r[i] = wave_max(r[i], part[(size_t)b * NPART + i]);
  }
#pragma unroll
  for (int i = 0; i < NPART; ++i) {
    for (int off = 32; off > 0; off >>= 1) r[i] = wave_max(r[i], __shfl_xor(r[i], off, 64));
  }
  if (blockDim.x > 64) {
    __shared__ double red[16][NPART];
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int i = 0; i < NPART; ++i) red[threadIdx.x >> 6][i] = r[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
#pragma unroll
        for (int i = 0; i < NPART; ++i) r[i] = wave_max(r[i], red[w][i]);
      }
    }
  }
  if (threadIdx.x != 0) return;
  if (kind == FIN_END_STAGE0) {
    step_end_body(ctl);
    kind = FIN_STAGE0;
  }
  if (kind != FIN_RHS && !ctl->active) return;
  const bool bad = !(r[0] < __builtin_huge_val());
  double sx = wave_max(r[0], r[2]), sy = wave_max(r[3], r[5]);
  if (sys == SYS_BUCKLEY) {
    sx = sy = bad ? 0.0 : buckley_max_speed(-r[1], r[0]);
    ctl->alpha[0][0] = sx;
    ctl->alpha[1][0] = sy;
  } else if (sys == SYS_EULER) {
    if (ph.lf_scalar) {
      for (int s = 0; s < 4; ++s) { ctl->alpha[0][s] = sx; ctl->alpha[1][s] = sy; }
    } else {
      ctl->alpha[0][0] = r[0]; ctl->alpha[0][1] = r[1]; ctl->alpha[0][2] = r[1]; ctl->alpha[0][3] = r[2];
      ctl->alpha[1][0] = r[3]; ctl->alpha[1][1] = r[4]; ctl->alpha[1][2] = r[4]; ctl->alpha[1][3] = r[5];
    }
  } else {
    ctl->alpha[0][0] = r[0];
    ctl->alpha[1][0] = r[3];
  }
  ctl->smax[0] = sx;
  ctl->smax[1] = sy;
  if (bad) {
    if (!ctl->bad) ctl->bad_step = ctl->steps;
    ctl->bad = 1;
    if (kind != FIN_RHS) ctl->active = 0;
    return;
  }
  if (kind == FIN_STAGE0) {
    if (ctl->max_steps > 0 && ctl->steps >= ctl->max_steps) { ctl->active = 0; return; }
    if (ctl->t >= ctl->t_final) { ctl->active = 0; return; }
    double dt;
    if (ctl->dt_fixed > 0.0) {
      dt = ctl->dt_fixed;
    } else if (ph.dt_rule == 1) {
      const double h = dim == 2 ? fmin(g.dx, g.dy) : g.dx;
      dt = ph.cfl * h * h;
    } else if (dim == 1) {
      dt = ph.cfl * g.dx / sx;
    } else {
      dt = ph.cfl / (sx / g.dx + sy / g.dy);
    }
    ctl->last = 0;
    if (ctl->t + dt >= ctl->t_final) { dt = ctl->t_final - ctl->t; ctl->last = 1; }
    ctl->dt = dt;
  }
}

template <int M>
__global__ __launch_bounds__(256) void k_wave_final(const double* __restrict__ part, int nblk, DevCtl* ctl,
                                                   Geom g, Phys ph, int dim, int kind, int sys) {
  wave_final_body(part, nblk, ctl, g, ph, dim, kind, sys);
}


static __global__ void k_step_end(DevCtl* ctl) { step_end_body(ctl); }

// Fixed-order FP64 sums of each component (deterministic for a given size):
// block b sums the contiguous chunk [b*chunk, (b+1)*chunk) with a fixed tree.
static __global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ q, size_t n, size_t chunk,
                                                     double* __restrict__ part) {
  const size_t lo = (size_t)blockIdx.x * chunk;
  const size_t hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += q[i];
  __shared__ double sm[256];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

}  // namespace za
