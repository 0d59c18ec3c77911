/*
 * WENO-ZA6 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of what the
 * MI355X path computes.  It exists so that the GPU library can be checked
 * against something written straight from the paper (Gu, Wang, Don, Jung,
 * "A Family of Even-Order Central-Upwind WENO Schemes with Averaged Downwind
 * and Novel Global Smoothness Indicators", arXiv 2603.26272).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * Everything is templated on the arithmetic type:
 *   double      -- the reference for FP64 parity,
 *   float       -- the FP32-reconstruction reading (state and RK3 stay FP64),
 *   __float128  -- the critical-point operator test (Section 3.1, tables
 *                  tab:ncp0 / tab:ncp1 print errors below FP64 rounding),
 *   Cnt         -- a counting scalar that tallies the algorithmic FLOPs.
 *
 * Build: g++ -O2 -ffp-contract=off -fPIC -shared -fopenmp  (see build.py).
 * -ffp-contract=off keeps every product and sum separately rounded, so the
 * results follow the written formulas operation by operation.
 *
 * Readings of the paper that are not stated in it (each listed in the design
 * notes of the repository):
 *   - weights are the non-affine-invariant Z type (mu = 1) unless the Ai flag
 *     is set (Section 3 says WENO-ZA6 uses Z weights without the Ai property);
 *   - Lax-Friedrichs speeds for systems are per characteristic field,
 *     alpha_s = max |lambda_s| over the interior cells of the RHS input;
 *   - the averaged state for the characteristic projection is Roe's average;
 *   - 2D time step: dt = CFL / (max(|u|+c)/dx + max(|v|+c)/dy);
 *   - initial data and the solution are point values at cell centres.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <memory>
#include <vector>
#include <algorithm>
#include <quadmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 quad;

/* ------------------------------------------------------------------------ */
/* FLOP-counting scalar.                                                     */
/* Every +,-,*,/,sqrt on data is counted once.  Operations a compiler folds   */
/* away are not counted: both operands literal constants, a product with a    */
/* literal 0 or +-1, or a sum with a literal 0.  |x|, max and comparisons are */
/* tallied separately and are not FLOPs.                                      */
/* ------------------------------------------------------------------------ */
struct OpCount { long long add, mul, div, sqrt, other; };
static OpCount g_ops;

struct Cnt {
  double v; bool lit;
  Cnt() : v(0), lit(true) {}
  Cnt(double x) : v(x), lit(true) {}           /* literal constant */
  static Cnt data(double x) { Cnt c(x); c.lit = false; return c; }
};
static inline Cnt mk(double v, bool lit) { Cnt c(v); c.lit = lit; return c; }
static inline bool is_lit(const Cnt& a, double x) { return a.lit && a.v == x; }
static inline Cnt operator+(Cnt a, Cnt b) {
  if (a.lit && b.lit) return mk(a.v + b.v, true);
  if (is_lit(a, 0.0)) return b;
  if (is_lit(b, 0.0)) return a;
  g_ops.add++; return mk(a.v + b.v, false);
}
static inline Cnt operator-(Cnt a) { return mk(-a.v, a.lit); }
static inline Cnt operator-(Cnt a, Cnt b) {
  if (a.lit && b.lit) return mk(a.v - b.v, true);
  if (is_lit(b, 0.0)) return a;
  if (is_lit(a, 0.0)) return mk(-b.v, false);
  g_ops.add++; return mk(a.v - b.v, false);
}
static inline Cnt operator*(Cnt a, Cnt b) {
  if (a.lit && b.lit) return mk(a.v * b.v, true);
  if (is_lit(a, 0.0) || is_lit(b, 0.0)) return mk(0.0, true);
  if (is_lit(a, 1.0)) return b;
  if (is_lit(b, 1.0)) return a;
  if (is_lit(a, -1.0)) return mk(-b.v, false);
  if (is_lit(b, -1.0)) return mk(-a.v, false);
  g_ops.mul++; return mk(a.v * b.v, false);
}
static inline Cnt operator/(Cnt a, Cnt b) {
  if (a.lit && b.lit) return mk(a.v / b.v, true);
  if (is_lit(a, 0.0)) return mk(0.0, true);
  if (is_lit(b, 1.0)) return a;
  g_ops.div++; return mk(a.v / b.v, false);
}
static inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
static inline bool operator<(Cnt a, Cnt b) { g_ops.other++; return a.v < b.v; }
static inline bool operator>(Cnt a, Cnt b) { g_ops.other++; return a.v > b.v; }
static inline bool operator<=(Cnt a, Cnt b) { g_ops.other++; return a.v <= b.v; }
static inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }

/* ---- per-type elementary functions ---- */
static inline double r_abs(double x) { return std::fabs(x); }
static inline float  r_abs(float x)  { return std::fabs(x); }
static inline quad   r_abs(quad x)   { return fabsq(x); }
static inline Cnt    r_abs(Cnt x)    { g_ops.other++; return mk(std::fabs(x.v), x.lit); }
static inline double r_sqrt(double x) { return std::sqrt(x); }
static inline float  r_sqrt(float x)  { return std::sqrt(x); }
static inline quad   r_sqrt(quad x)   { return sqrtq(x); }
static inline Cnt    r_sqrt(Cnt x)    { if (!x.lit) g_ops.sqrt++; return mk(std::sqrt(x.v), x.lit); }
static inline double r_pow(double x, double p) { return std::pow(x, p); }
static inline float  r_pow(float x, float p)   { return std::pow(x, p); }
static inline quad   r_pow(quad x, quad p)     { return powq(x, p); }
static inline Cnt    r_pow(Cnt x, Cnt p)       { g_ops.other++; return mk(std::pow(x.v, p.v), false); }
static inline double r_exp(double x) { return std::exp(x); }
static inline quad   r_exp(quad x)   { return expq(x); }
template <class R> static inline R r_max(R a, R b) { return (a < b) ? b : a; }

template <class R> static inline R lit(double x) { return R(x); }
template <class R> static inline R frac(int n, int d) { return R(n) / R(d); }
/* state (double) -> arithmetic type */
template <class R> static inline R from_state(double x) { return R(x); }
template <> inline Cnt from_state<Cnt>(double x) { return Cnt::data(x); }
template <class R> static inline double to_state(R x) { return (double)x; }
template <> inline double to_state<Cnt>(Cnt x) { return x.v; }
template <> inline double to_state<quad>(quad x) { return (double)x; }

/* ------------------------------------------------------------------------ */
/* O1: one split reconstruction at one interface (Section 2, Section 3).     */
/* ------------------------------------------------------------------------ */
struct ReconParams {
  double p;        /* power parameter p of eq:weight_nonlinear (paper: 1) */
  double eps;      /* sensitivity epsilon (paper: 1e-40 in FP64)          */
  int ai;          /* 1: affine-invariant descaler mu[f] of eq:aimu       */
  double mu0;      /* mu_0 of eq:aimu                                      */
  int linear;      /* 1: omega = d (the linear sixth-order central flux)   */
  int alt_tau = 0; /* 1: the alternative indicator tau' of eq:GSI_alt      */
  double L = 1.0;  /* L and q of eq:weights_unnormalized (paper: 1, 1)   */
  double q = 1.0;
};

/* Unnormalised weight alpha_k / d_k = (L + Gamma_k)^q of
 * eq:weights_unnormalized with Gamma_k = (tau / bden)^p (eq:weight_nonlinear),
 * bden = beta_k + eps mu^2.  Reading for L = 0: alpha_k = d_k tau^(pq) /
 * bden^(pq); the factor (tau / bmin)^(pq) (bmin the smallest bden of the
 * stencil) is common to every k and cancels in omega_k (eq:weights_general),
 * so alpha_k / d_k is taken as (bmin / bden)^(pq) <= 1: omega stays defined
 * where tau = 0 (the limit tau -> 0+, JS-type weights) and nothing overflows. */
template <class R>
static R z_alpha(R tau, R bden, R bmin, const ReconParams& P) {
  if (P.L == 0.0) {
    R a = bmin / bden;
    if (P.p * P.q != 1.0) a = r_pow(a, R(P.p * P.q));
    return a;
  }
  R g = tau / bden;
  if (P.p != 1.0) g = r_pow(g, R(P.p));
  R a = R(P.L) + g;
  if (P.q != 1.0) a = r_pow(a, R(P.q));
  return a;
}

/* Constants of the r = 3 scheme, built in the arithmetic type R so that the
 * quad build carries them to quad accuracy.  Values as printed in Section 3:
 * c6 (central flux), c_k (eq:subflux_S6_coeffs), d (ideal weights),
 * c_tau (eq:GSI with r = 3). */
template <class R> struct ZA6Const {
  R c6[6];
  R ck[4][3];
  R d[4];
  R ctau[6];
  R half, thirteen_thirds, quarter;
  ZA6Const() {
    const int c6n[6] = {1, -8, 37, 37, -8, 1};
    for (int j = 0; j < 6; ++j) c6[j] = frac<R>(c6n[j], 60);
    const int ckn[4][3] = {{2, -7, 11}, {-1, 5, 2}, {2, 5, -1}, {11, -7, 2}};
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 3; ++j) ck[k][j] = frac<R>(ckn[k][j], 6);
    const int dn[4] = {1, 9, 9, 1};
    for (int k = 0; k < 4; ++k) d[k] = frac<R>(dn[k], 20);
    const int ctn[6] = {-1, 5, -10, 10, -5, 1};
    for (int j = 0; j < 6; ++j) ctau[j] = R(ctn[j]);
    half = frac<R>(1, 2);
    thirteen_thirds = frac<R>(13, 3);
    quarter = frac<R>(1, 4);
  }
};

/* Intermediate values of one reconstruction, exported for the tests. */
struct ReconDetail {
  double q[4];      /* candidate fluxes q_0..q_3                        */
  double beta[5];   /* beta_0, beta_1, beta_2, beta_d, beta_3 (average)  */
  double tau;       /* global smoothness indicator                      */
  double mu;        /* descaler (1 unless Ai)                           */
  double omega[4];  /* nonlinear weights                                */
};

/* Reconstruct h at x_{i+1/2} from v[0..5] = (f_{i-2}, ..., f_{i+3}).
 * For the negative split flux the caller passes the same six points in
 * reversed order (mirror symmetry about x_{i+1/2}, Section 2).            */
template <class R>
static R recon_za6(const R v[6], const ZA6Const<R>& K, const ReconParams& P,
                   ReconDetail* det) {
  /* Candidate fluxes: q_k = <c_k, f_k> on S_k = {x_{i-2+k}, .., x_{i+k}}
   * (eq:numerical_subflux with the coefficients eq:subflux_S6_coeffs). */
  R q[4];
  for (int k = 0; k < 4; ++k)
    q[k] = K.ck[k][0] * v[k] + K.ck[k][1] * v[k + 1] + K.ck[k][2] * v[k + 2];

  R out;
  if (P.linear) {
    /* omega = d: the convex combination collapses to the linear flux
     * (eq:numerical_flux_FD_linear_comb). */
    out = K.d[0] * q[0] + K.d[1] * q[1] + K.d[2] * q[2] + K.d[3] * q[3];
    if (det) {
      for (int k = 0; k < 4; ++k) { det->q[k] = to_state(q[k]); det->omega[k] = to_state(K.d[k]); }
      for (int k = 0; k < 5; ++k) det->beta[k] = 0;
      det->tau = 0; det->mu = 1;
    }
    return out;
  }

  /* Local smoothness indicators, eq:SI written out for r = 3.  With dx = 1
   * and x_i = 0, the quadratic p_k on S_k (cells at offsets o, o+1, o+2,
   * o = k-2) has p_k'' = 2 a_2 with a_2 = (f_o - 2 f_{o+1} + f_{o+2}) / 2
   * and p_k'(0) = a_1 = (f_{o+1} - f_o) - (2o+1) a_2 (the cell averages of
   * xi and xi^2 over [l-1/2, l+1/2] are l and l^2 + 1/12).  eq:SI then gives
   * beta = a_1^2 + (13/3) a_2^2.  k = 3 is the downwind polynomial p_3, whose
   * indicator beta_d is measured over I_i like the others. */
  R beta[4];
  for (int k = 0; k < 4; ++k) {
    const int o = k - 2;
    R a2 = K.half * (v[k] - lit<R>(2.0) * v[k + 1] + v[k + 2]);
    R a1 = (v[k + 1] - v[k]) - lit<R>((double)(2 * o + 1)) * a2;
    beta[k] = a1 * a1 + K.thirteen_thirds * (a2 * a2);
  }
  /* beta_3: arithmetic mean of beta_0, beta_1, beta_2 and beta_d
   * (eq:SI_downwind with r = 3). */
  R beta_d = beta[3];
  R beta3 = K.quarter * (beta[0] + beta[1] + beta[2] + beta_d);
  R b[4] = {beta[0], beta[1], beta[2], beta3};

  /* Global smoothness indicator tau = <c_tau, f^6>^2 (eq:GSI), or the
   * alternative tau' = (13/12) <c_tau, f^6>^2 + <c'_tau, f^6>^2 with
   * c'_tau = (1, -4, 6, -4, 1, 0) (eq:GSI_alt, the remark after eq:GSI). */
  R t = R(0);
  for (int j = 0; j < 6; ++j) t = t + K.ctau[j] * v[j];
  R tau = t * t;
  if (P.alt_tau) {
    const int ctp[6] = {1, -4, 6, -4, 1, 0};
    R t4 = R(0);
    for (int j = 0; j < 6; ++j) t4 = t4 + lit<R>((double)ctp[j]) * v[j];
    tau = frac<R>(13, 12) * tau + t4 * t4;
  }

  /* Descaler mu[f] (eq:aimu); mu = 1 for the non-Ai Z weights. */
  R mu = R(1);
  if (P.ai) {
    R mean = R(0);
    for (int j = 0; j < 6; ++j) mean = mean + v[j];
    mean = mean / R(6);
    R s = R(0);
    for (int j = 0; j < 6; ++j) s = s + r_abs(v[j] - mean);
    mu = s / R(6) + R(P.mu0);
  }

  /* Gamma_k (eq:weight_nonlinear), alpha_k = d_k (L + Gamma_k)^q
   * (eq:weights_unnormalized; the paper's runs: L = q = 1), omega_k
   * (eq:weights_general). */
  const R eps = R(P.eps);
  const R epsmu2 = P.ai ? eps * (mu * mu) : eps;
  R bden[4];
  for (int k = 0; k < 4; ++k) bden[k] = b[k] + epsmu2;
  R bmin = bden[0];
  if (P.L == 0.0)
    for (int k = 1; k < 4; ++k) bmin = bden[k] < bmin ? bden[k] : bmin;
  R alpha[4], asum = R(0);
  for (int k = 0; k < 4; ++k) {
    alpha[k] = K.d[k] * z_alpha<R>(tau, bden[k], bmin, P);
    asum = asum + alpha[k];
  }
  R omega[4];
  for (int k = 0; k < 4; ++k) omega[k] = alpha[k] / asum;

  /* eq:numerical_flux_WENO */
  out = omega[0] * q[0] + omega[1] * q[1] + omega[2] * q[2] + omega[3] * q[3];

  if (det) {
    for (int k = 0; k < 4; ++k) { det->q[k] = to_state(q[k]); det->omega[k] = to_state(omega[k]); }
    det->beta[0] = to_state(beta[0]); det->beta[1] = to_state(beta[1]);
    det->beta[2] = to_state(beta[2]); det->beta[3] = to_state(beta_d);
    det->beta[4] = to_state(beta3);
    det->tau = to_state(tau); det->mu = to_state(mu);
  }
  return out;
}

/* ------------------------------------------------------------------------ */
/* O1 for any even order 2r (Section 2, Section 3, Appendix A).              */
/* The tables are exact rationals derived from the definitions by            */
/* oracle/coeffs.py (pinned there against the printed tables) and handed     */
/* over once per order through orc_set_order_tables.                         */
/* ------------------------------------------------------------------------ */
enum { R_MAX = 6 };
struct GenTab { int set; std::vector<long long> num, den; };
static GenTab g_gen[R_MAX + 1];

template <class R> struct GenConst {
  int r;
  R ck[R_MAX + 1][R_MAX];                 /* c_k on S_k, k = 0..r            */
  R d[R_MAX + 1];                         /* ideal weights                   */
  R ctau[2 * R_MAX];                      /* (2r-1)-th difference            */
  R D[R_MAX + 1][R_MAX][R_MAX][R_MAX];    /* D[k][l][m][j]: coefficient of   */
                                          /* xi^m in p_k^(l), from f_j       */
  R I[2 * R_MAX];                         /* int_{-1/2}^{1/2} xi^s           */
  explicit GenConst(int rr) : r(rr) {
    const GenTab& T = g_gen[rr];
    size_t at = 0;
    auto next = [&]() { R v = R((double)T.num[at]) / R((double)T.den[at]); ++at; return v; };
    for (int k = 0; k <= r; ++k)
      for (int j = 0; j < r; ++j) ck[k][j] = next();
    for (int k = 0; k <= r; ++k) d[k] = next();
    for (int j = 0; j < 2 * r; ++j) ctau[j] = next();
    for (int k = 0; k <= r; ++k)
      for (int l = 1; l < r; ++l)
        for (int m = 0; m < r - l; ++m)
          for (int j = 0; j < r; ++j) D[k][l][m][j] = next();
    for (int s2 = 0; s2 <= 2 * r - 4; ++s2) I[s2] = next();
  }
};

/* Reconstruct h at x_{i+1/2} from v[0..2r-1] = (f_{i-r+1}, .., f_{i+r}).
 * det (optional) receives q[0..r], beta_0..beta_{r-1}, beta_d, beta_r (the
 * mean), tau, mu, omega[0..r]: 3r + 6 values. */
template <class R>
static R recon_gen(const R* v, const GenConst<R>& K, const ReconParams& P, double* det) {
  const int r = K.r;
  /* candidates q_k = <c_k, f_k>, S_k = cells i-r+1+k .. i+k */
  R q[R_MAX + 1];
  for (int k = 0; k <= r; ++k) {
    R acc = R(0);
    for (int j = 0; j < r; ++j) acc = acc + K.ck[k][j] * v[k + j];
    q[k] = acc;
  }
  R out = R(0);
  if (P.linear) {
    for (int k = 0; k <= r; ++k) out = out + K.d[k] * q[k];
    return out;
  }
  /* eq:SI: beta = sum_l int_{I_i} (p_k^(l))^2, written with the
   * coefficients a_m of p_k^(l) (linear in f) and the interval moments. */
  R beta[R_MAX + 2];
  for (int k = 0; k <= r; ++k) {
    R b = R(0);
    for (int l = 1; l < r; ++l) {
      R a[R_MAX];
      const int nm = r - l;
      for (int m = 0; m < nm; ++m) {
        R acc = R(0);
        for (int j = 0; j < r; ++j) acc = acc + K.D[k][l][m][j] * v[k + j];
        a[m] = acc;
      }
      for (int m1 = 0; m1 < nm; ++m1)
        for (int m2 = 0; m2 < nm; ++m2)
          if ((m1 + m2) % 2 == 0) b = b + K.I[m1 + m2] * (a[m1] * a[m2]);
    }
    beta[k] = b;
  }
  /* beta[r] is beta_d; the downwind substencil takes the mean of the r
   * upwind indicators and beta_d (eq:SI_downwind) */
  R sum = R(0);
  for (int k = 0; k <= r; ++k) sum = sum + beta[k];
  const R beta_d = beta[r];
  const R beta_r = sum / R(r + 1);
  R bw[R_MAX + 1];
  for (int k = 0; k < r; ++k) bw[k] = beta[k];
  bw[r] = beta_r;
  /* tau = <c_tau, f^{2r}>^2 (eq:GSI) */
  R t = R(0);
  for (int j = 0; j < 2 * r; ++j) t = t + K.ctau[j] * v[j];
  const R tau = t * t;
  R mu = R(1);
  if (P.ai) {
    R mean = R(0);
    for (int j = 0; j < 2 * r; ++j) mean = mean + v[j];
    mean = mean / R(2 * r);
    R sa = R(0);
    for (int j = 0; j < 2 * r; ++j) sa = sa + r_abs(v[j] - mean);
    mu = sa / R(2 * r) + R(P.mu0);
  }
  const R eps = R(P.eps);
  const R epsmu2 = P.ai ? eps * (mu * mu) : eps;
  R bden[R_MAX + 1];
  for (int k = 0; k <= r; ++k) bden[k] = bw[k] + epsmu2;
  R bmin = bden[0];
  if (P.L == 0.0)
    for (int k = 1; k <= r; ++k) bmin = bden[k] < bmin ? bden[k] : bmin;
  R alpha[R_MAX + 1], asum = R(0);
  for (int k = 0; k <= r; ++k) {
    alpha[k] = K.d[k] * z_alpha<R>(tau, bden[k], bmin, P);
    asum = asum + alpha[k];
  }
  R omega[R_MAX + 1];
  for (int k = 0; k <= r; ++k) {
    omega[k] = alpha[k] / asum;
    out = out + omega[k] * q[k];
  }
  if (det) {
    int o = 0;
    for (int k = 0; k <= r; ++k) det[o++] = to_state(q[k]);
    for (int k = 0; k < r; ++k) det[o++] = to_state(beta[k]);
    det[o++] = to_state(beta_d);
    det[o++] = to_state(beta_r);
    det[o++] = to_state(tau);
    det[o++] = to_state(mu);
    for (int k = 0; k <= r; ++k) det[o++] = to_state(omega[k]);
  }
  return out;
}

/* The scheme of one sweep: r = 3 takes the sixth-order routine above,
 * other orders the generic one. */
template <class R> struct Scheme {
  int r;
  ZA6Const<R> k6;
  const GenConst<R>* kg;
  R operator()(const R* v, const ReconParams& P) const {
    return r == 3 ? recon_za6<R>(v, k6, P, nullptr) : recon_gen<R>(v, *kg, P, nullptr);
  }
};

/* Owns the generic tables of one order in type R (built before any parallel
 * region, read-only inside). */
template <class R> struct SchemeFor {
  std::unique_ptr<GenConst<R>> g;
  Scheme<R> S;
  explicit SchemeFor(int r) {
    if (r != 3) g.reset(new GenConst<R>(r));
    S.r = r;
    S.kg = g.get();
  }
};

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own; mirrors the library's fields).     */
/* ------------------------------------------------------------------------ */
enum { SYS_ADVECTION = 0, SYS_EULER = 1, SYS_BURGERS = 2, SYS_BUCKLEY = 3 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };
enum { DT_CFL = 0, DT_CFL_H2 = 1 };
enum { LF_PER_FIELD = 0, LF_SCALAR = 1 };

extern "C" {
typedef struct {
  int32_t dim, system, nx, ny;
  double xlo, xhi, ylo, yhi;
  int32_t bc_x, bc_y;
  double gamma;
  double adv_speed[2];
  double cfl;
  int32_t dt_rule;
  int32_t recon_fp32;
  double p, eps;
  int32_t ai;
  double mu0;
  int32_t lf;
  int32_t linear_weights;
  int32_t order;          /* r of the order-2r scheme (0 or 3: WENO-ZA6) */
  int32_t pp_limiter;     /* 1: positivity-preserving flux limiter in steps */
  int32_t alt_tau;        /* 1: tau' of eq:GSI_alt instead of tau (r = 3)   */
  double weight_L, weight_q; /* L, q of eq:weights_unnormalized (0, 0: 1, 1) */
} orc_problem;
}

static int ncomp(const orc_problem& P) {
  if (P.system == SYS_EULER) return P.dim == 1 ? 3 : 4;
  return 1;
}

/* Ghost cells (three per side, the width of the six-point stencil):
 * periodic wraps, transmissive copies the nearest interior cell. */
static inline int bc_index(int j, int n, int bc) {
  if (bc == BC_PERIODIC) { int r = j % n; return r < 0 ? r + n : r; }
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

/* ------------------------------------------------------------------------ */
/* Scalar flux functions (Section 2, Section 4.1).                            */
/* ------------------------------------------------------------------------ */
template <class R> static R scalar_flux(const orc_problem& P, int dir, R u) {
  switch (P.system) {
    case SYS_ADVECTION: return from_state<R>(P.adv_speed[dir]) * u;
    case SYS_BURGERS: return R(0.5) * u * u;
    default: { /* Buckley-Leverett, tab:scalar_fluxes */
      R a = u * u, w = R(1) - u;
      return a / (a + R(0.25) * (w * w));
    }
  }
}
static double scalar_dflux(const orc_problem& P, int dir, double u) {
  switch (P.system) {
    case SYS_ADVECTION: return P.adv_speed[dir];
    case SYS_BURGERS: return u;
    default: {
      /* f = u^2 / D, D = u^2 + (1-u)^2/4,  f' = (2u D - u^2 D') / D^2 */
      double D = u * u + 0.25 * (1 - u) * (1 - u);
      double Dp = 2 * u - 0.5 * (1 - u);
      return (2 * u * D - u * u * Dp) / (D * D);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Euler: primitive variables, physical flux, wave speeds, eigenvectors.     */
/* Fields (rho, rho u, [rho v], E); p = (gamma-1)(E - rho |u|^2 / 2).         */
/* ------------------------------------------------------------------------ */
template <class R>
static void euler_flux(int m, int dir, R gm1, const R* Q, R* F) {
  R rho = Q[0];
  R u = Q[1] / rho;
  if (m == 3) {
    R p = gm1 * (Q[2] - R(0.5) * rho * u * u);
    F[0] = Q[1];
    F[1] = Q[1] * u + p;
    F[2] = (Q[2] + p) * u;
    return;
  }
  R v = Q[2] / rho;
  R p = gm1 * (Q[3] - R(0.5) * rho * (u * u + v * v));
  R un = dir == 0 ? u : v;
  F[0] = rho * un;
  F[1] = Q[1] * un + (dir == 0 ? p : R(0));
  F[2] = Q[2] * un + (dir == 1 ? p : R(0));
  F[3] = (Q[3] + p) * un;
}

/* Left/right eigenvectors of dF_dir/dQ at a state (u, v, H, c).  Columns of
 * Rm are right eigenvectors for the eigenvalues (u_n - c, u_n, [u_n], u_n + c);
 * Lm is the inverse (rows are left eigenvectors).  Textbook forms, written
 * out separately for each direction. */
template <class R>
static void euler_eigen(int m, int dir, R gm1, R u, R v, R H, R c, R* Rm, R* Lm) {
  const R q2 = m == 3 ? R(0.5) * (u * u) : R(0.5) * (u * u + v * v);
  const R b1 = gm1 / (c * c);
  const R b2 = b1 * q2;
  const R ic = R(1) / c;
  const R h = R(0.5);
  if (m == 3) {
    R Rv[9] = {R(1), R(1), R(1),
               u - c, u, u + c,
               H - u * c, q2, H + u * c};
    R Lv[9] = {h * (b2 + u * ic), -h * (b1 * u + ic), h * b1,
               R(1) - b2, b1 * u, -b1,
               h * (b2 - u * ic), -h * (b1 * u - ic), h * b1};
    for (int i = 0; i < 9; ++i) { Rm[i] = Rv[i]; Lm[i] = Lv[i]; }
    return;
  }
  if (dir == 0) {
    R Rv[16] = {R(1), R(1), R(0), R(1),
                u - c, u, R(0), u + c,
                v, v, R(1), v,
                H - u * c, q2, v, H + u * c};
    R Lv[16] = {h * (b2 + u * ic), -h * (b1 * u + ic), -h * (b1 * v), h * b1,
                R(1) - b2, b1 * u, b1 * v, -b1,
                -v, R(0), R(1), R(0),
                h * (b2 - u * ic), -h * (b1 * u - ic), -h * (b1 * v), h * b1};
    for (int i = 0; i < 16; ++i) { Rm[i] = Rv[i]; Lm[i] = Lv[i]; }
  } else {
    R Rv[16] = {R(1), R(0), R(1), R(1),
                u, R(1), u, u,
                v - c, R(0), v, v + c,
                H - v * c, u, q2, H + v * c};
    R Lv[16] = {h * (b2 + v * ic), -h * (b1 * u), -h * (b1 * v + ic), h * b1,
                -u, R(1), R(0), R(0),
                R(1) - b2, b1 * u, b1 * v, -b1,
                h * (b2 - v * ic), -h * (b1 * u), -h * (b1 * v - ic), h * b1};
    for (int i = 0; i < 16; ++i) { Rm[i] = Rv[i]; Lm[i] = Lv[i]; }
  }
}

/* Roe-averaged interface state of two neighbouring cells L, R (the state
 * whose eigenvectors the characteristic-wise splitting of Section 4.2 uses;
 * the paper does not name the average, Roe's is the standard one):
 *   w_L = sqrt(rho_L) / (sqrt(rho_L) + sqrt(rho_R)),  w_R = 1 - w_L (formed
 *   as sqrt(rho_R) / (..)),  u~ = w_L u_L + w_R u_R (also v~ and the total
 *   enthalpy H~ = (E + p)/rho),  c~^2 = (gamma-1)(H~ - |u~|^2/2).
 * For this state A(Q~) (Q_R - Q_L) = F(Q_R) - F(Q_L) holds exactly, in both
 * directions of a 2D sweep, which the tests check. */
template <class R>
static void roe_state(int m, R gm1, const R* QL, const R* QR, R* u_out, R* v_out, R* H_out, R* c_out) {
  const R h = R(0.5);
  R rl = QL[0], rr = QR[0];
  R ul = QL[1] / rl, ur = QR[1] / rr;
  R vl = m == 4 ? QL[2] / rl : R(0), vr = m == 4 ? QR[2] / rr : R(0);
  R pl = gm1 * (QL[m - 1] - h * rl * (ul * ul + vl * vl));
  R pr = gm1 * (QR[m - 1] - h * rr * (ur * ur + vr * vr));
  R Hl = (QL[m - 1] + pl) / rl, Hr = (QR[m - 1] + pr) / rr;
  R sl = r_sqrt(rl), sr = r_sqrt(rr);
  R wl = sl / (sl + sr), wr = sr / (sl + sr);
  R u = wl * ul + wr * ur;
  R v = wl * vl + wr * vr;
  R H = wl * Hl + wr * Hr;
  R q2 = m == 4 ? h * (u * u + v * v) : h * (u * u);
  R c2 = gm1 * (H - q2);
  *u_out = u; *v_out = v; *H_out = H;
  *c_out = r_sqrt(c2);
}

/* Wave speeds of one sweep direction over the interior cells, in FP64:
 * alpha[s] = max |lambda_s| (s over the m characteristic fields) and
 * smax = max(|u_n| + c).  Returns 0 if the state is finite and physical,
 * 1 otherwise (rho <= 0, p <= 0 or a non-finite value). */
/* Largest |f'(u)| of the Buckley-Leverett flux over u in [lo, hi].  f' =
 * u (1-u) / (2 D^2), D = u^2 + (1-u)^2/4, has its extrema where
 * (1-2u) D = 2 u (1-u) D', i.e. at the roots of 10 u^3 - 15 u^2 + 1 (one in
 * each of (-1/2, 0), (0, 1/2), (1, 3/2)); the maximum over an interval is at
 * an end point or at such a root inside it. */
static double buckley_max_speed(double lo, double hi) {
  auto fp = [](double u) { double D = u * u + 0.25 * (1 - u) * (1 - u); return 0.5 * u * (1 - u) / (D * D); };
  auto cubic = [](double u) { return (10 * u - 15) * u * u + 1; };
  double best = std::max(std::fabs(fp(lo)), std::fabs(fp(hi)));
  const double brackets[3][2] = {{-0.5, 0.0}, {0.0, 0.5}, {1.0, 1.5}};
  for (int b = 0; b < 3; ++b) {
    double a = brackets[b][0], c = brackets[b][1];
    const bool rising = cubic(a) < 0;
    for (int it = 0; it < 200 && a < c; ++it) {     /* bisection to the last bit */
      double mid = 0.5 * (a + c);
      if (mid <= a || mid >= c) break;
      if ((cubic(mid) < 0) == rising) a = mid; else c = mid;
    }
    const double root = a;
    if (root > lo && root < hi) best = std::max(best, std::fabs(fp(root)));
  }
  return best;
}

static int wave_speeds(const orc_problem& P, const double* q, int dir, double* alpha, double* smax) {
  const int m = ncomp(P);
  const size_t ncell = (size_t)P.nx * P.ny;
  int bad = 0;
  for (int s = 0; s < 4; ++s) alpha[s] = 0;
  *smax = 0;
  if (P.system == SYS_BUCKLEY) {
    /* non-convex flux: the LF speed is max |f'| over the range of the data
     * (the data's own values can all sit where f' vanishes, e.g. u in {0, 1}) */
    double lo = INFINITY, hi = -INFINITY;
    for (size_t i = 0; i < ncell; ++i) {
      double u = q[i];
      if (u != u) bad = 1;
      lo = std::min(lo, u);
      hi = std::max(hi, u);
    }
    double a = bad ? 0.0 : buckley_max_speed(lo, hi);
    alpha[0] = a; *smax = a;
    return bad;
  }
  if (P.system != SYS_EULER) {
    double a = 0;
    for (size_t i = 0; i < ncell; ++i) {
      double u = q[i];
      if (u != u) bad = 1;
      a = std::max(a, std::fabs(scalar_dflux(P, dir, u)));
    }
    alpha[0] = a; *smax = a;
    return bad;
  }
  const double gm1 = P.gamma - 1;
  for (size_t i = 0; i < ncell; ++i) {
    double Q[4];
    for (int c = 0; c < m; ++c) Q[c] = q[c * ncell + i];
    double rho = Q[0];
    double u = Q[1] / rho, v = m == 4 ? Q[2] / rho : 0.0;
    double E = Q[m - 1];
    double p = gm1 * (E - 0.5 * rho * (u * u + v * v));
    double c2 = P.gamma * p / rho;
    if (!(rho > 0) || !(p > 0) || !(c2 > 0) || !std::isfinite(E) || !std::isfinite(Q[1])) { bad = 1; continue; }
    double c = std::sqrt(c2);
    double un = dir == 0 ? u : v;
    alpha[0] = std::max(alpha[0], std::fabs(un - c));
    alpha[1] = std::max(alpha[1], std::fabs(un));
    alpha[m - 1] = std::max(alpha[m - 1], std::fabs(un + c));
    *smax = std::max(*smax, std::fabs(un) + c);
  }
  if (m == 4) alpha[2] = alpha[1];
  if (P.lf == LF_SCALAR) {
    for (int s = 0; s < m; ++s) alpha[s] = *smax;
  }
  return bad;
}

/* ------------------------------------------------------------------------ */
/* O2/O3: numerical fluxes of one sweep.                                      */
/* Interface k (0..n) of a line of n cells sits at x_{k-1/2}, between cells   */
/* k-1 and k; its 2r-point stencil is cells k-r .. k+r-1.                     */
/* ------------------------------------------------------------------------ */
template <class R>
static void line_fluxes(const orc_problem& P, const Scheme<R>& S, const ReconParams& RP,
                        int dir, const double* alpha, int n, int bc,
                        /* gather cell j (ghosts allowed) of this line into Q[m] */
                        const double* const* lineptr, size_t stride,
                        double* Fhat /* [m][n+1], stride n+1 */) {
  const int m = ncomp(P);
  const int r = S.r, w = 2 * r;
  const R h = R(0.5);
  /* physical flux of every cell including r ghosts per side, f_j = f(Q_j) */
  std::vector<R> Qc((size_t)(n + 2 * r) * m), Fc((size_t)(n + 2 * r) * m);
  for (int j = -r; j < n + r; ++j) {
    int jj = bc_index(j, n, bc);
    R* Qj = &Qc[(size_t)(j + r) * m];
    R* Fj = &Fc[(size_t)(j + r) * m];
    for (int c = 0; c < m; ++c) Qj[c] = from_state<R>(lineptr[c][(size_t)jj * stride]);
    if (P.system == SYS_EULER) euler_flux<R>(m, dir, R(P.gamma - 1), Qj, Fj);
    else Fj[0] = scalar_flux<R>(P, dir, Qj[0]);
  }
  R vp[2 * R_MAX], vm[2 * R_MAX];
  for (int k = 0; k <= n; ++k) {
    if (P.system != SYS_EULER) {
      /* Global Lax-Friedrichs splitting f^(+-) = (f +- alpha Q)/2 (eq:LF),
       * f^+ reconstructed from (f_{i-r+1..i+r}), f^- from the mirrored
       * stencil (f_{i+r..i-r+1}); F = f^+ + f^-. */
      R a = from_state<R>(alpha[0]);
      for (int j = 0; j < w; ++j) {
        const int cj = k - r + j;
        R Qj = Qc[(size_t)(cj + r)], Fj = Fc[(size_t)(cj + r)];
        vp[j] = h * (Fj + a * Qj);
        vm[w - 1 - j] = h * (Fj - a * Qj);
      }
      R fh = S(vp, RP) + S(vm, RP);
      Fhat[k] = to_state(fh);
      continue;
    }
    /* Characteristic-wise LF splitting for the Euler system (Section 4.2):
     * Roe average of cells k-1 and k, project the 2r-point stencil of Q and
     * F onto the characteristic fields, split and reconstruct each field,
     * project back. */
    const R gm1 = R(P.gamma - 1);
    R u, v, H, c;
    roe_state<R>(m, gm1, &Qc[(size_t)(k - 1 + r) * m], &Qc[(size_t)(k + r) * m], &u, &v, &H, &c);
    R Rm[16], Lm[16];
    euler_eigen<R>(m, dir, gm1, u, v, H, c, Rm, Lm);
    R W[2 * R_MAX][4], G[2 * R_MAX][4];
    for (int j = 0; j < w; ++j) {
      const R* Qj = &Qc[(size_t)(k - r + j + r) * m];
      const R* Fj = &Fc[(size_t)(k - r + j + r) * m];
      for (int s2 = 0; s2 < m; ++s2) {
        R wv = R(0), g = R(0);
        for (int cc = 0; cc < m; ++cc) {
          wv = wv + Lm[s2 * m + cc] * Qj[cc];
          g = g + Lm[s2 * m + cc] * Fj[cc];
        }
        W[j][s2] = wv; G[j][s2] = g;
      }
    }
    R gh[4];
    for (int s2 = 0; s2 < m; ++s2) {
      R a = from_state<R>(alpha[s2]);
      for (int j = 0; j < w; ++j) {
        vp[j] = h * (G[j][s2] + a * W[j][s2]);
        vm[w - 1 - j] = h * (G[j][s2] - a * W[j][s2]);
      }
      gh[s2] = S(vp, RP) + S(vm, RP);
    }
    for (int cc = 0; cc < m; ++cc) {
      R f = R(0);
      for (int s2 = 0; s2 < m; ++s2) f = f + Rm[cc * m + s2] * gh[s2];
      Fhat[(size_t)cc * (n + 1) + k] = to_state(f);
    }
  }
}

struct Ctx {
  orc_problem P;
  ReconParams RP;
  int m;
  int r;          /* order 2r of the scheme */
  double dx, dy;
  size_t ncell;
};

static int make_ctx(const orc_problem* p, Ctx* C) {
  if (!p) return 1;
  C->P = *p;
  if (p->dim != 1 && p->dim != 2) return 1;
  if (p->nx < 1 || p->ny < 1 || (p->dim == 1 && p->ny != 1)) return 1;
  C->m = ncomp(*p);
  C->r = p->order == 0 ? 3 : p->order;
  if (C->r < 2 || C->r > R_MAX) return 1;
  if (C->r != 3 && !g_gen[C->r].set) return 1;   /* tables not handed over */
  C->RP.p = p->p; C->RP.eps = p->eps; C->RP.ai = p->ai; C->RP.mu0 = p->mu0;
  C->RP.linear = p->linear_weights;
  C->RP.alt_tau = p->alt_tau;
  if (p->alt_tau && C->r != 3) return 1;
  if (p->weight_L == 0.0 && p->weight_q == 0.0) { C->RP.L = 1.0; C->RP.q = 1.0; }
  else { C->RP.L = p->weight_L; C->RP.q = p->weight_q; }
  if (!(C->RP.L >= 0.0) || !(C->RP.q >= 1.0)) return 1;
  C->dx = (p->xhi - p->xlo) / p->nx;
  C->dy = p->dim == 2 ? (p->yhi - p->ylo) / p->ny : 1.0;
  C->ncell = (size_t)p->nx * p->ny;
  return 0;
}

/* All numerical fluxes of one direction for state q: fx [m][ny][nx+1] or
 * fy [m][ny+1][nx].  alpha from this RHS's own input. */
template <class R>
static int sweep_fluxes(const Ctx& C, const double* q, int dir, const double* alpha, double* F) {
  const orc_problem& P = C.P;
  const int m = C.m;
  const int nx = P.nx, ny = P.ny;
  const SchemeFor<R> SF(C.r);
  const Scheme<R>& K = SF.S;
  if (dir == 0) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
      const double* lp[4];
      for (int c = 0; c < m; ++c) lp[c] = q + c * C.ncell + (size_t)y * nx;
      std::vector<double> Fl((size_t)m * (nx + 1));
      line_fluxes<R>(P, K, C.RP, 0, alpha, nx, P.bc_x, lp, 1, Fl.data());
      for (int c = 0; c < m; ++c)
        for (int k = 0; k <= nx; ++k)
          F[(size_t)c * ny * (nx + 1) + (size_t)y * (nx + 1) + k] = Fl[(size_t)c * (nx + 1) + k];
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int x = 0; x < nx; ++x) {
      const double* lp[4];
      for (int c = 0; c < m; ++c) lp[c] = q + c * C.ncell + x;
      std::vector<double> Fl((size_t)m * (ny + 1));
      line_fluxes<R>(P, K, C.RP, 1, alpha, ny, P.bc_y, lp, (size_t)nx, Fl.data());
      for (int c = 0; c < m; ++c)
        for (int k = 0; k <= ny; ++k)
          F[(size_t)c * (ny + 1) * nx + (size_t)k * nx + x] = Fl[(size_t)c * (ny + 1) + k];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Positivity-preserving flux limiter for the Euler equations, after Hu,     */
/* Adams and Shu (J. Comput. Phys. 242, 2013), which the paper cites for its */
/* shock-diffraction test (Section 4.3).  A forward-Euler stage with step dt */
/* is a convex combination of one-dimensional updates, and each cell's      */
/* update of one direction is the mean of two "half" states, one per face:  */
/*   U_i - 2 mu F_{i+1/2}  and  U_{i+1} + 2 mu F_{i+1/2},                   */
/* mu = dt S / s_dir with s_dir = max(|u_n| + c) of that direction and     */
/* S = sum over directions of s_d / dx_d (1D: mu = dt/dx).  With the first- */
/* order global Lax-Friedrichs flux in place of F both half states stay     */
/* positive whenever dt S <= 1/2.  Each face's flux becomes                  */
/*   F~ = F_LF + theta (F - F_LF),                                           */
/* theta in [0, 1] the largest value (up to the bounds below) that keeps    */
/* density and pressure of both half states >= eps = 1e-13: density is      */
/* linear in theta (exact bound); pressure is concave in the state, so the  */
/* chord from the LF half state to the density-limited one is a lower bound */
/* and gives theta_p in closed form.  Faces whose high-order half states are */
/* admissible keep theta = 1.  Only stages (with a dt) are limited.          */
/* ------------------------------------------------------------------------ */
static const double PP_EPS = 1e-13;

static double pp_pressure(int m, double gm1, const double* U) {
  double k = U[1] * U[1];
  if (m == 4) k += U[2] * U[2];
  return gm1 * (U[m - 1] - 0.5 * k / U[0]);
}

/* theta keeping A + theta B admissible (A: the LF half state) */
static double pp_theta(int m, double gm1, const double* A, const double* B) {
  const double rA = A[0], pA = (rA > 0) ? pp_pressure(m, gm1, A) : -1.0;
  if (!(rA >= PP_EPS) || !(pA >= PP_EPS)) return 0.0;
  double th = 1.0;
  const double r1 = rA + B[0];
  if (r1 < PP_EPS) th = (rA - PP_EPS) / (rA - r1);
  double U1[4];
  for (int c = 0; c < m; ++c) U1[c] = A[c] + th * B[c];
  const double p1 = pp_pressure(m, gm1, U1);
  if (p1 < PP_EPS) th = th * (pA - PP_EPS) / (pA - p1);
  return th;
}

/* Limit the interface fluxes F of direction dir of state q in place. */
static void pp_limit(const Ctx& C, const double* q, int dir, double dt, double S, double s_dir, double* F) {
  const orc_problem& P = C.P;
  const int m = C.m, nx = P.nx, ny = P.ny;
  const double gm1 = P.gamma - 1.0;
  const double mu = dt * S / s_dir;
  const int n = dir == 0 ? nx : ny, lines = dir == 0 ? ny : nx;
  const int bc = dir == 0 ? P.bc_x : P.bc_y;
#pragma omp parallel for schedule(static)
  for (int l = 0; l < lines; ++l) {
    for (int k = 0; k <= n; ++k) {
      const int jl = bc_index(k - 1, n, bc), jr = bc_index(k, n, bc);
      const size_t il = dir == 0 ? (size_t)l * nx + jl : (size_t)jl * nx + l;
      const size_t ir = dir == 0 ? (size_t)l * nx + jr : (size_t)jr * nx + l;
      double QL[4], QR[4], FL[4], FR[4], Fh[4], Flf[4];
      for (int c = 0; c < m; ++c) { QL[c] = q[c * C.ncell + il]; QR[c] = q[c * C.ncell + ir]; }
      euler_flux<double>(m, dir, gm1, QL, FL);
      euler_flux<double>(m, dir, gm1, QR, FR);
      const size_t fi = dir == 0 ? (size_t)l * (nx + 1) + k : (size_t)k * nx + l;
      const size_t fs = dir == 0 ? (size_t)ny * (nx + 1) : (size_t)(ny + 1) * nx;
      double AL[4], BL[4], AR[4], BR[4];
      for (int c = 0; c < m; ++c) {
        Fh[c] = F[c * fs + fi];
        Flf[c] = 0.5 * (FL[c] + FR[c] - s_dir * (QR[c] - QL[c]));
        AL[c] = QL[c] - 2.0 * mu * Flf[c];
        BL[c] = -2.0 * mu * (Fh[c] - Flf[c]);
        AR[c] = QR[c] + 2.0 * mu * Flf[c];
        BR[c] = 2.0 * mu * (Fh[c] - Flf[c]);
      }
      const double th = std::min(pp_theta(m, gm1, AL, BL), pp_theta(m, gm1, AR, BR));
      if (th < 1.0)
        for (int c = 0; c < m; ++c) F[c * fs + fi] = Flf[c] + th * (Fh[c] - Flf[c]);
    }
  }
}

/* L(Q) = -(F_{i+1/2} - F_{i-1/2})/dx  [+ the same in y]   (eq:hyperbolic_1D_scalar_h,
 * dimension by dimension in 2D, Section 4.3).  dt > 0 with the limiter on:
 * the fluxes of the stage Q + dt L(Q) are limited first. */
template <class R>
static int rhs_impl(const Ctx& C, const double* q, double* rhs, double dt = 0.0) {
  const orc_problem& P = C.P;
  const int m = C.m, nx = P.nx, ny = P.ny;
  double ax[4], ay[4], sx, sy = 0;
  int bad = wave_speeds(P, q, 0, ax, &sx);
  if (P.dim == 2) bad |= wave_speeds(P, q, 1, ay, &sy);
  const bool pp = P.pp_limiter && P.system == SYS_EULER && dt > 0 && !bad;
  const double S = sx / C.dx + (P.dim == 2 ? sy / C.dy : 0.0);
  std::vector<double> fx((size_t)m * ny * (nx + 1));
  sweep_fluxes<R>(C, q, 0, ax, fx.data());
  if (pp) pp_limit(C, q, 0, dt, S, sx, fx.data());
  for (int c = 0; c < m; ++c)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const double* f = &fx[(size_t)c * ny * (nx + 1) + (size_t)y * (nx + 1)];
        rhs[(size_t)c * C.ncell + (size_t)y * nx + x] = -(f[x + 1] - f[x]) / C.dx;
      }
  if (P.dim == 2) {
    std::vector<double> fy((size_t)m * (ny + 1) * nx);
    sweep_fluxes<R>(C, q, 1, ay, fy.data());
    if (pp) pp_limit(C, q, 1, dt, S, sy, fy.data());
    for (int c = 0; c < m; ++c)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const double* f = &fy[(size_t)c * (ny + 1) * nx];
          rhs[(size_t)c * C.ncell + (size_t)y * nx + x] += -(f[(size_t)(y + 1) * nx + x] - f[(size_t)y * nx + x]) / C.dy;
        }
  }
  return bad;
}

static int rhs_any(const Ctx& C, const double* q, double* rhs, double dt = 0.0) {
  return C.P.recon_fp32 ? rhs_impl<float>(C, q, rhs, dt) : rhs_impl<double>(C, q, rhs, dt);
}

/* CFL time step from the current state (Section 4, reading for 2D). */
static double cfl_dt(const Ctx& C, const double* q, int* bad) {
  const orc_problem& P = C.P;
  if (P.dt_rule == DT_CFL_H2) {
    double h = P.dim == 2 ? std::min(C.dx, C.dy) : C.dx;
    return P.cfl * h * h;
  }
  double a[4], sx, sy = 0;
  *bad |= wave_speeds(P, q, 0, a, &sx);
  if (P.dim == 1) return P.cfl * C.dx / sx;
  *bad |= wave_speeds(P, q, 1, a, &sy);
  return P.cfl / (sx / C.dx + sy / C.dy);
}

/* One SSP-RK3 step in Shu-Osher form:
 *   Q1 = Qn + dt L(Qn)
 *   Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1))
 *   Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2))                                     */
static int rk3_step(const Ctx& C, double* q, double dt) {
  const size_t n = (size_t)C.m * C.ncell;
  std::vector<double> L(n), q1(n), q2(n);
  int bad = rhs_any(C, q, L.data(), dt);
  for (size_t i = 0; i < n; ++i) q1[i] = q[i] + dt * L[i];
  bad |= rhs_any(C, q1.data(), L.data(), dt);
  for (size_t i = 0; i < n; ++i) q2[i] = 0.75 * q[i] + 0.25 * (q1[i] + dt * L[i]);
  bad |= rhs_any(C, q2.data(), L.data(), dt);
  for (size_t i = 0; i < n; ++i) q[i] = (1.0 / 3.0) * q[i] + (2.0 / 3.0) * (q2[i] + dt * L[i]);
  for (size_t i = 0; i < n; ++i) if (!std::isfinite(q[i])) bad = 1;
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Section 3.1 critical-point operator test: f(x) = x^(ncp+1) e^(0.75 x) on   */
/* nodes x_j = -1 + j dx, j = 0..2/dx; D_j = (h_{j+1/2} - h_{j-1/2})/dx with  */
/* the positive reconstruction; error = max_j |D_j - f'(x_j)|.                */
/* ------------------------------------------------------------------------ */
template <class R>
static double critical_point_test(int ncp, int inv_dx, double p, int eps_mode, double eps, int ai, double mu0) {
  static const ZA6Const<R> K;
  const int n = 2 * inv_dx;              /* nodes 0..n */
  const R dx = R(2) / R(n);
  ReconParams RP;
  RP.p = p; RP.ai = ai; RP.mu0 = mu0; RP.linear = 0;
  if (eps_mode == 1) {
    /* epsilon = dx^(2(ncp-1)) (tab:ncp1, ncp = 4, 5) */
    R e = R(1);
    for (int i = 0; i < 2 * (ncp - 1); ++i) e = e * dx;
    RP.eps = (double)e;
    /* keep the quad value exact enough: eps only enters as beta + eps */
  } else {
    RP.eps = eps;
  }
  auto f = [&](R x) { R r = R(1); for (int i = 0; i < ncp + 1; ++i) r = r * x; return r * r_exp(R(0.75) * x); };
  auto fp = [&](R x) {
    R xn = R(1); for (int i = 0; i < ncp; ++i) xn = xn * x;   /* x^ncp */
    return (R(ncp + 1) * xn + R(0.75) * xn * x) * r_exp(R(0.75) * x);
  };
  /* interfaces j+1/2 for j = -1 .. n need nodes j-2 .. j+3, i.e. -3 .. n+3 */
  std::vector<R> fv((size_t)n + 7);
  for (int j = -3; j <= n + 3; ++j) fv[(size_t)(j + 3)] = f(R(-1) + R(j) * dx);
  std::vector<R> fh((size_t)n + 2);
  for (int j = -1; j <= n; ++j) {
    R v[6];
    for (int t = 0; t < 6; ++t) v[t] = fv[(size_t)(j - 2 + t + 3)];
    fh[(size_t)(j + 1)] = recon_za6<R>(v, K, RP, nullptr);
  }
  R err = R(0);
  for (int j = 0; j <= n; ++j) {
    R D = (fh[(size_t)(j + 1)] - fh[(size_t)j]) / dx;
    R e = r_abs(D - fp(R(-1) + R(j) * dx));
    if (err < e) err = e;
  }
  return (double)err;
}

/* ------------------------------------------------------------------------ */
/* C ABI of the oracle (loaded by the test-suite through ctypes).            */
/* ------------------------------------------------------------------------ */
extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* O1 in FP64 on v[0..5]; detail (15 doubles: q[4], beta[5], tau, mu,
 * omega[4]) may be NULL. */
double orc_recon(const double* v6, double p, double eps, int ai, double mu0, int linear, double* detail) {
  static const ZA6Const<double> K;
  ReconParams RP{p, eps, ai, mu0, linear};
  ReconDetail d;
  double r = recon_za6<double>(v6, K, RP, detail ? &d : nullptr);
  if (detail) std::memcpy(detail, &d, sizeof(d));
  return r;
}
/* As orc_recon with the weight parameters L and q of eq:weights_unnormalized. */
double orc_recon_lq(const double* v6, double p, double eps, int ai, double mu0, double L, double q,
                    double* detail) {
  static const ZA6Const<double> K;
  ReconParams RP{p, eps, ai, mu0, 0};
  RP.L = L; RP.q = q;
  ReconDetail d;
  double r = recon_za6<double>(v6, K, RP, detail ? &d : nullptr);
  if (detail) std::memcpy(detail, &d, sizeof(d));
  return r;
}
/* As orc_recon with the alternative global indicator tau' (eq:GSI_alt). */
double orc_recon_alt(const double* v6, double p, double eps, int ai, double mu0, double* detail) {
  static const ZA6Const<double> K;
  ReconParams RP{p, eps, ai, mu0, 0};
  RP.alt_tau = 1;
  ReconDetail d;
  double r = recon_za6<double>(v6, K, RP, detail ? &d : nullptr);
  if (detail) std::memcpy(detail, &d, sizeof(d));
  return r;
}
/* O1 in FP32 (inputs rounded to float first). */
double orc_recon_f32(const double* v6, double p, double eps, int ai, double mu0, int linear) {
  static const ZA6Const<float> K;
  ReconParams RP{p, eps, ai, mu0, linear};
  float v[6];
  for (int j = 0; j < 6; ++j) v[j] = (float)v6[j];
  return (double)recon_za6<float>(v, K, RP, nullptr);
}
/* O1 in quad precision; the six inputs are given as decimal strings so that
 * the test can supply values beyond FP64 resolution. */
double orc_recon_q(const char* const* v6, double p, double eps, int ai, double mu0, char* out, int outlen) {
  static const ZA6Const<quad> K;
  ReconParams RP{p, eps, ai, mu0, 0};
  quad v[6];
  for (int j = 0; j < 6; ++j) v[j] = strtoflt128(v6[j], nullptr);
  quad r = recon_za6<quad>(v, K, RP, nullptr);
  if (out) quadmath_snprintf(out, (size_t)outlen, "%.36Qe", r);
  return (double)r;
}

double orc_critical_point_test(int ncp, int inv_dx, double p, int eps_mode, double eps, int ai, double mu0, int use_quad) {
  if (use_quad) return critical_point_test<quad>(ncp, inv_dx, p, eps_mode, eps, ai, mu0);
  return critical_point_test<double>(ncp, inv_dx, p, eps_mode, eps, ai, mu0);
}

/* Eigenvector matrices used by the characteristic projection (row-major
 * m x m), exported so the tests can check L R = I and L A R = diag(lambda). */
void orc_euler_eigen(int m, int dir, double gamma, double u, double v, double H, double c,
                     double* Rm, double* Lm) {
  euler_eigen<double>(m, dir, gamma - 1, u, v, H, c, Rm, Lm);
}

int orc_ncomp(const orc_problem* p) { return ncomp(*p); }

/* The Roe-averaged interface state (u~, v~, H~, c~) of two cells, as the
 * interface fluxes use it (m = 3: 1D, v~ = 0; m = 4: 2D, either sweep
 * direction, since the average does not depend on it). */
void orc_roe_state(int m, double gamma, const double* QL, const double* QR, double* out4) {
  double u, v, H, c;
  roe_state<double>(m, gamma - 1.0, QL, QR, &u, &v, &H, &c);
  out4[0] = u; out4[1] = v; out4[2] = H; out4[3] = c;
}

int orc_wave_speeds(const orc_problem* p, const double* q, double* alpha /*[2][4]*/, double* smax /*[2]*/) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  int bad = wave_speeds(C.P, q, 0, alpha, &smax[0]);
  if (C.P.dim == 2) bad |= wave_speeds(C.P, q, 1, alpha + 4, &smax[1]);
  else { for (int s = 0; s < 4; ++s) alpha[4 + s] = 0; smax[1] = 0; }
  return bad ? 4 : 0;
}

/* Tables of the order-2r scheme as n exact rationals num[i]/den[i], in the
 * layout of oracle/coeffs.py flat_rationals(r).  Returns 0 on success. */
int orc_set_order_tables(int r, const int64_t* num, const int64_t* den, int n) {
  if (r < 2 || r > R_MAX || !num || !den) return 1;
  const int expect = (r + 1) * r + (r + 1) + 2 * r + (r + 1) * (r * (r - 1) / 2) * r + (2 * r - 3);
  if (n != expect) return 1;
  GenTab& T = g_gen[r];
  T.num.assign(num, num + n);
  T.den.assign(den, den + n);
  for (int i = 0; i < n; ++i) if (T.den[i] == 0) return 1;
  T.set = 1;
  return 0;
}

/* One reconstruction of the order-2r scheme from v[0..2r-1] in FP64 (fp32 =
 * 0), FP32 (1) or quad (2, result rounded to FP64); detail (FP64 path only,
 * may be NULL) receives 3r + 6 values: q_0..q_r, beta_0..beta_{r-1}, beta_d,
 * beta_r, tau, mu, omega_0..omega_r. */
double orc_recon_r(int r, const double* v, double p, double eps, int ai, double mu0, int linear,
                   int prec, double* detail) {
  if (r < 2 || r > R_MAX || !g_gen[r].set) return NAN;
  ReconParams RP; RP.p = p; RP.eps = eps; RP.ai = ai; RP.mu0 = mu0; RP.linear = linear;
  if (prec == 1) {
    GenConst<float> K(r);
    float x[2 * R_MAX];
    for (int j = 0; j < 2 * r; ++j) x[j] = (float)v[j];
    return (double)recon_gen<float>(x, K, RP, nullptr);
  }
  if (prec == 2) {
    GenConst<quad> K(r);
    quad x[2 * R_MAX];
    for (int j = 0; j < 2 * r; ++j) x[j] = (quad)v[j];
    return (double)recon_gen<quad>(x, K, RP, nullptr);
  }
  GenConst<double> K(r);
  return recon_gen<double>(v, K, RP, detail);
}

/* orc_recon_r (FP64) with the weight parameters L and q. */
double orc_recon_r_lq(int r, const double* v, double p, double eps, int ai, double mu0, double L, double q,
                      double* detail) {
  if (r < 2 || r > R_MAX || !g_gen[r].set) return NAN;
  ReconParams RP; RP.p = p; RP.eps = eps; RP.ai = ai; RP.mu0 = mu0; RP.linear = 0;
  RP.L = L; RP.q = q;
  GenConst<double> K(r);
  return recon_gen<double>(v, K, RP, detail);
}

/* Interface fluxes: fx [m][ny][nx+1]; fy [m][ny+1][nx] (2D only, may be NULL). */
int orc_fluxes(const orc_problem* p, const double* q, double* fx, double* fy) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  double a[4], s;
  int bad = wave_speeds(C.P, q, 0, a, &s);
  if (C.P.recon_fp32) sweep_fluxes<float>(C, q, 0, a, fx); else sweep_fluxes<double>(C, q, 0, a, fx);
  if (C.P.dim == 2 && fy) {
    bad |= wave_speeds(C.P, q, 1, a, &s);
    if (C.P.recon_fp32) sweep_fluxes<float>(C, q, 1, a, fy); else sweep_fluxes<double>(C, q, 1, a, fy);
  }
  return bad ? 4 : 0;
}

/* Fluxes of selected lines only (spot checks at full size): dir 0 gives the
 * x-interface fluxes of rows lines[0..nl-1] as out[l][m][nx+1]; dir 1 the
 * y-interface fluxes of columns lines[..] as out[l][m][ny+1].  The LF speeds
 * are the global ones of q, exactly as in orc_fluxes. */
int orc_fluxes_lines(const orc_problem* p, const double* q, int dir, const int* lines, int nl, double* out) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  const orc_problem& P = C.P;
  double a[4], s;
  int bad = wave_speeds(P, q, dir, a, &s);
  const int n = dir == 0 ? P.nx : P.ny;
  const int m = C.m;
  const SchemeFor<float> SF32(C.r);
  const SchemeFor<double> SF64(C.r);
#pragma omp parallel for schedule(dynamic)
  for (int l = 0; l < nl; ++l) {
    const double* lp[4];
    for (int c = 0; c < m; ++c)
      lp[c] = dir == 0 ? q + c * C.ncell + (size_t)lines[l] * P.nx : q + c * C.ncell + lines[l];
    const size_t stride = dir == 0 ? 1 : (size_t)P.nx;
    double* o = out + (size_t)l * m * (n + 1);
    if (P.recon_fp32) {
      line_fluxes<float>(P, SF32.S, C.RP, dir, a, n, dir == 0 ? P.bc_x : P.bc_y, lp, stride, o);
    } else {
      line_fluxes<double>(P, SF64.S, C.RP, dir, a, n, dir == 0 ? P.bc_x : P.bc_y, lp, stride, o);
    }
  }
  return bad ? 4 : 0;
}

int orc_rhs(const orc_problem* p, const double* q, double* rhs) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  return rhs_any(C, q, rhs) ? 4 : 0;
}

double orc_cfl_dt(const orc_problem* p, const double* q) {
  Ctx C; if (make_ctx(p, &C)) return -1;
  int bad = 0;
  return cfl_dt(C, q, &bad);
}

/* One RK3 step; dt <= 0 takes the CFL step. */
int orc_step(const orc_problem* p, double* q, double dt, double* dt_used) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  int bad = 0;
  if (!(dt > 0)) dt = cfl_dt(C, q, &bad);
  if (dt_used) *dt_used = dt;
  bad |= rk3_step(C, q, dt);
  return bad ? 4 : 0;
}

/* Integrate to t_final.  Fixed-step rule (CFL*h^2): n = ceil(T/dt (1-1e-12))
 * steps, the last one T - (n-1) dt.  CFL rule: recompute dt each step from
 * the current state and clip the last step to T.  t_final <= 0 runs exactly
 * max_steps CFL steps without clipping.  max_steps > 0 caps the count. */
int orc_solve(const orc_problem* p, double* q, double t_final, int64_t max_steps,
              int64_t* steps_out, double* t_out) {
  Ctx C; if (make_ctx(p, &C)) return 1;
  int bad = 0;
  int64_t steps = 0;
  double t = 0;
  if (t_final > 0 && C.P.dt_rule == DT_CFL_H2) {
    double dt = cfl_dt(C, q, &bad);
    int64_t n = (int64_t)std::ceil(t_final / dt * (1 - 1e-12));
    for (int64_t s = 0; s < n; ++s) {
      if (max_steps > 0 && steps >= max_steps) break;
      double h = (s == n - 1) ? t_final - (double)(n - 1) * dt : dt;
      bad |= rk3_step(C, q, h);
      t = (s == n - 1) ? t_final : t + h;
      ++steps;
      if (bad) break;
    }
  } else if (t_final > 0) {
    while (t < t_final) {
      if (max_steps > 0 && steps >= max_steps) break;
      double dt = cfl_dt(C, q, &bad);
      if (bad) break;
      bool last = false;
      if (t + dt >= t_final) { dt = t_final - t; last = true; }
      bad |= rk3_step(C, q, dt);
      t = last ? t_final : t + dt;
      ++steps;
      if (bad) break;
    }
  } else {
    for (int64_t s = 0; s < max_steps; ++s) {
      double dt = cfl_dt(C, q, &bad);
      if (bad) break;
      bad |= rk3_step(C, q, dt);
      t += dt;
      ++steps;
      if (bad) break;
    }
  }
  if (steps_out) *steps_out = steps;
  if (t_out) *t_out = t;
  return bad ? 4 : 0;
}

/* Algorithmic operation counts of the interface fluxes of one RHS
 * evaluation, via the counting scalar.  dir_mask bit 0: x-sweep, bit 1:
 * y-sweep (2D).  counts[0..4] = add/sub, mul, div, sqrt, other (abs, max,
 * compare, pow).  The physical flux is evaluated once per cell of each line
 * including its six ghost cells; the caller separates per-cell and
 * per-interface work by counting two sizes.  Returns the number of interface
 * reconstructions counted, or -1 on error.  The wave-speed reduction, the
 * flux difference and the RK3 combination are FP64 closed forms, counted by
 * the caller. */
int64_t orc_count_ops(const orc_problem* p, const double* q, int dir_mask, int64_t* counts) {
  Ctx C; if (make_ctx(p, &C)) return -1;
#ifdef _OPENMP
  int saved = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  const orc_problem& P = C.P;
  double ax[4], ay[4], s;
  wave_speeds(P, q, 0, ax, &s);
  wave_speeds(P, q, 1, ay, &s);
  std::memset(&g_ops, 0, sizeof(g_ops));
  int64_t nir = 0;
  if (dir_mask & 1) {
    std::vector<double> fx((size_t)C.m * P.ny * (P.nx + 1));
    sweep_fluxes<Cnt>(C, q, 0, ax, fx.data());
    nir += (int64_t)(P.nx + 1) * P.ny;
  }
  if (P.dim == 2 && (dir_mask & 2)) {
    std::vector<double> fy((size_t)C.m * (P.ny + 1) * P.nx);
    sweep_fluxes<Cnt>(C, q, 1, ay, fy.data());
    nir += (int64_t)P.nx * (P.ny + 1);
  }
  counts[0] = g_ops.add; counts[1] = g_ops.mul; counts[2] = g_ops.div;
  counts[3] = g_ops.sqrt; counts[4] = g_ops.other;
#ifdef _OPENMP
  omp_set_num_threads(saved);
#endif
  return nir;
}

} /* extern "C" */
