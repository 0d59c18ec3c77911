// Device building blocks of the WENO-ZA6 right-hand side for gfx950.
//
// Paper: Gu, Wang, Don, Jung, "A Family of Even-Order Central-Upwind WENO
// Schemes with Averaged Downwind and Novel Global Smoothness Indicators"
// (arXiv 2603.26272).  Everything here is per interface and lives in
// registers: the six-point stencil, the Roe-averaged eigenvectors, the four
// candidate fluxes, the smoothness indicators and the weights.
//
// Arithmetic type T is double (FP64 path) or float (FP32 reconstruction);
// the state is always double.
#pragma once
#include <hip/hip_runtime.h>

#include "za_order_tables.hpp"
#include <stdint.h>

namespace za {

// ---------------------------------------------------------------------------
// Parameters of the nonlinear weights (eq:weight_nonlinear, eq:aimu), already
// rescaled for the exact power-of-two scaling used below.
// ---------------------------------------------------------------------------
template <class T>
struct WeightCfg {
  T eps16;    // 16 epsilon   (Z weights, indicators of 2v scaled by 4)
  T eps6;     // 6 epsilon    (Z weights from differences, za6_diff)
  T eps6q;    // 6 epsilon / 4 (its downwind indicator, kept at a quarter)
  T eps4;     // 4 epsilon    (Ai weights after dividing by mu(2v)^2;
              //               order-2r Z weights on 2v)
  T eps1;     // epsilon      (order-2r Ai weights after dividing by mu(2v)^2)
  T mu0x2;    // 2 mu_0       (descaler of 2v)
  T p;        // power parameter (1 on the fast path)
  int ai;     // 1: affine-invariant descaler
  int linear; // 1: omega = d
  int alt_tau; // 1: tau' of eq:GSI_alt (r = 3, general weights)
  T L;        // L of eq:weights_unnormalized (1 on the fast path)
  T q;        // q of eq:weights_unnormalized (1 on the fast path)
  T pq;       // p q (the exponent when L = 0)
};

// Weight variants compiled as separate kernels: the paper's Z weights with
// p = 1 and mu = 1 (the fast path), or everything else (Ai descaler, p != 1,
// linear weights) decided at run time.
enum { WV_Z1 = 0, WV_GENERAL = 1 };

// The hardware FP64 reciprocal and reciprocal-square-root estimates are
// good to a relative 2^-24 (measured over 4M normal operands on gfx950: at
// most 4.6e-8 and 5.2e-8).  One refinement squares that error: the
// reciprocal takes one Newton-Raphson step (r <- r + r (1 - x r)), the
// quotient one residual correction of a r (q <- q + r (a - x q)), each
// within about 2^-48 relative, three orders of magnitude inside the flux
// tolerance of 1e-12.  Operands stay far from the denormal and overflow
// ranges here (positive normal densities and weight sums >= 1e-276), so no
// exponent scaling is needed.
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double div_nr(double a, double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double q = a * r;
  return fma(fma(-x, q, a), r, q);
}
__device__ __forceinline__ float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float div_nr(float a, float x) { return a * __builtin_amdgcn_rcpf(x); }

// Square root s and half reciprocal square root h = 1/(2 sqrt(x)) of a
// positive normal number together: the hardware reciprocal-square-root
// estimate refined by one coupled Goldschmidt iteration (e = 1/2 - h s,
// s <- s + s e, h <- h + h e), which squares its relative error (to about
// 2^-48 in FP64, the FP32 rounding in FP32).
__device__ __forceinline__ void sqrt_rsq(double x, double& s, double& h) {
  const double r = __builtin_amdgcn_rsq(x);
  s = x * r;
  h = 0.5 * r;
  const double e = fma(-h, s, 0.5);
  s = fma(s, e, s);
  h = fma(h, e, h);
}
__device__ __forceinline__ void sqrt_rsq(float x, float& s, float& h) {
  const float r = __builtin_amdgcn_rsqf(x);
  s = x * r;
  h = 0.5f * r;
  const float e = fmaf(-h, s, 0.5f);
  s = fmaf(s, e, s);
  h = fmaf(h, e, h);
}

// alpha_k / d_k = (L + Gamma_k)^q (eq:weights_unnormalized), Gamma_k =
// (tau / b)^p (eq:weight_nonlinear), b = beta_k + eps mu^2 on the common
// scale of the caller.  L = 0: tau^(pq) is common to every k and cancels in
// omega_k, and so does bmin^(-pq) (bmin the smallest b of the stencil), so the
// weight is taken as (bmin / b)^(pq) <= 1, defined where tau = 0 and free of
// overflow.  Outside WV_GENERAL this is the paper's 1 + tau / b.
template <class T, int WV>
__device__ __forceinline__ T z_alpha(T tau, T b, T bmin, const WeightCfg<T>& w) {
  if (WV == WV_GENERAL && w.L == T(0)) {
    T a = bmin * rcp_nr(b);
    if (w.pq != T(1)) a = pow(a, w.pq);
    return a;
  }
  T g = tau * rcp_nr(b);
  if (WV == WV_GENERAL && w.p != T(1)) g = pow(g, w.p);
  if (WV != WV_GENERAL) return T(1) + g;
  T a = w.L + g;
  if (w.q != T(1)) a = pow(a, w.q);
  return a;
}

// ---------------------------------------------------------------------------
// One WENO-ZA6 reconstruction at x_{i+1/2} (Section 3: r = 3).
//
// Input: s = (s0..s5) = 2 (f_{i-2}, .., f_{i+3}), i.e. twice the split flux
// values, which the caller forms with one FMA each (g +- alpha w).  Output:
// twice the reconstructed flux.  The negative split flux passes its six
// values in reverse order (mirror symmetry about x_{i+1/2}, Section 2).
//
//  candidates  q_k = <c_k, f_k>, c_k = (2,-7,11)/6, (-1,5,2)/6, (2,5,-1)/6,
//              (11,-7,2)/6                         (eq:subflux_S6_coeffs)
//  indicators  beta_k = (13/12) D2_k^2 + (1/4) D1_k^2: eq:SI for quadratics
//              (D2 the second difference, D1 twice the slope of p_k at x_i);
//              k = 3 is the downwind beta_d, measured on I_i.  This sum of
//              squares equals the printed quadratic forms <f_k, B_k f_k>
//              (eq:SI_S6) and is never negative.
//  downwind    beta_3 = (beta_0 + beta_1 + beta_2 + beta_d)/4 (eq:SI_downwind)
//  global      tau = <c_tau, f>^2 with <c_tau, f> the fifth difference
//              (c_tau = (-1,5,-10,10,-5,1), eq:GSI)
//  weights     alpha_k = d_k (1 + tau/(beta_k + eps mu^2)), d = (1,9,9,1)/20,
//              omega_k = alpha_k / sum alpha (eq:weights_unnormalized with
//              L = q = 1, p = 1; eq:weights_general)
//
// Exact rescaling.  With s = 2f the code forms B_k = (13/3) D2(s)^2 + D1(s)^2
// = 16 beta_k(f) and T = (2 D5(s))^2 = 16 tau(f); multiplying by powers of
// two is exact in binary floating point, so tau/(beta + eps) is evaluated as
// T/(B + 16 eps) with identical rounding.  (Ai: mu(s) = 2 mu(f) with 2 mu_0,
// then T/mu(s)^2 and B/mu(s)^2 are 4 tau/mu^2 and 4 beta/mu^2, so 4 eps.)
//
// This direct form serves the general weights; the paper's Z weights take
// za6_diff below (the other orders take zar).
// ---------------------------------------------------------------------------
template <class T, int WV>
__device__ __forceinline__ T za6(T s0, T s1, T s2, T s3, T s4, T s5, const WeightCfg<T>& w) {
  const T c13 = T(1) / T(3), c16 = T(1) / T(6), c56 = T(5) / T(6);
  // first and second differences; the candidates are written around the
  // centre values: q_0 = s2 + (5 d1 - 2 d0)/6, q_1 = s2 + (d1 + 2 d2)/6,
  // q_2 = s3 - (2 d2 + d3)/6, q_3 = s3 + (2 d4 - 5 d3)/6 (= <c_k, f_k>)
  const T d0 = s1 - s0, d1 = s2 - s1, d2 = s3 - s2, d3 = s4 - s3, d4 = s5 - s4;
  const T q0 = fma(c56, d1, fma(-c13, d0, s2));
  const T q1 = fma(c13, d2, fma(c16, d1, s2));
  const T q2 = fma(-c16, d3, fma(-c13, d2, s3));
  const T q3 = fma(c13, d4, fma(-c56, d3, s3));
  if (WV == WV_GENERAL && w.linear) {
    return (q0 + q3 + T(9) * (q1 + q2)) * T(0.05);
  }
  const T e0 = d1 - d0, e1 = d2 - d1, e2 = d3 - d2, e3 = d4 - d3;
  const T g0 = fma(T(3), d1, -d0);       // s0 - 4 s1 + 3 s2
  const T g1 = d1 + d2;                  // -(s1 - s3)
  const T g2 = fma(T(3), d2, -d3);       // -(3 s2 - 4 s3 + s4)
  const T g3 = fma(T(5), d3, T(-3) * d4);// -5 s3 + 8 s4 - 3 s5
  const T k133 = T(13) / T(3);
  const T t5 = (e3 - e0) + T(3) * (e1 - e2);   // fifth difference
  const T t2 = t5 + t5;
  T B0 = fma(k133 * e0, e0, g0 * g0);
  T B1 = fma(k133 * e1, e1, g1 * g1);
  T B2 = fma(k133 * e2, e2, g2 * g2);
  const T Bd = fma(k133 * e3, e3, g3 * g3);
  T B3 = T(0.25) * ((B0 + B1) + (B2 + Bd));
  T tau = t2 * t2;
  if (WV == WV_GENERAL && w.alt_tau) {
    // tau' = (13/12) <c_tau, f>^2 + <c'_tau, f>^2, c'_tau = (1,-4,6,-4,1,0):
    // with s = 2f, 16 tau' = (13/12) t2^2 + (2 (e0 - 2 e1 + e2))^2
    const T t4 = fma(T(-2), e1, e0 + e2);
    tau = fma(T(13.0 / 12.0), tau, T(4) * (t4 * t4));
  }
  T eps = w.eps16;
  if (WV == WV_GENERAL && w.ai) {
    const T mean = (s0 + s1 + s2 + s3 + s4 + s5) * c16;
    const T mu = (fabs(s0 - mean) + fabs(s1 - mean) + fabs(s2 - mean) + fabs(s3 - mean) +
                  fabs(s4 - mean) + fabs(s5 - mean)) * c16 + w.mu0x2;
    const T imu2 = rcp_nr(mu * mu);
    B0 *= imu2; B1 *= imu2; B2 *= imu2; B3 *= imu2; tau *= imu2;
    eps = w.eps4;
  }
  const T b0 = B0 + eps, b1 = B1 + eps, b2 = B2 + eps, b3 = B3 + eps;
  const T bmin = (WV == WV_GENERAL && w.L == T(0)) ? fmin(fmin(b0, b1), fmin(b2, b3)) : T(0);
  const T a0 = z_alpha<T, WV>(tau, b0, bmin, w), a1 = T(9) * z_alpha<T, WV>(tau, b1, bmin, w),
          a2 = T(9) * z_alpha<T, WV>(tau, b2, bmin, w), a3 = z_alpha<T, WV>(tau, b3, bmin, w);
  return div_nr(fma(a0, q0, fma(a1, q1, fma(a2, q2, a3 * q3))), (a0 + a1) + (a2 + a3));
}

// ---------------------------------------------------------------------------
// WENO-ZA6 with the paper's Z weights (p = 1, L = q = 1), evaluated from
// the first differences d_j = s_{j+1} - s_j (j = 0..4) of s = 2 (f_{i-2}, ..,
// f_{i+3}) and measured from the anchor value s_A (A = 2 or 3): returns
// 3 (R - s_A), R twice the reconstructed flux as in za6.  Since the weights
// sum to one, R - s_A = sum_k omega_k (q_k - s_A), and 3 (q_k - s_A) has
// short coefficients in the d's, one or two FMAs each:
//   A = 2:  2.5 d1 - d0,  0.5 d1 + d2,  2 d2 - 0.5 d3,  3 d2 - 2.5 d3 + d4
//   A = 3:  2.5 d1 - d0 - 3 d2,  0.5 d1 - 2 d2,  -d2 - 0.5 d3,  d4 - 2.5 d3
// (eq:subflux_S6_coeffs written around s_A).
//
// Indicators.  With e and g the second differences and twice the slopes of
// za6, 6 beta_k(f) = (3/8) ((13/3) e_k^2 + g_k^2) (eq:SI_S6 with s = 2f) is a
// positive definite quadratic form in the two differences (u, w) = (d_k,
// d_{k+1}) of its stencil, 5 w^2 - 5.5 u w + 2 u^2 (k = 0), 2 w^2 - 2.5 u w +
// 2 u^2 (k = 1), 2 w^2 - 5.5 u w + 5 u^2 (k = 2) and 5 w^2 - 14.5 u w + 11 u^2
// (downwind candidate on I_i), and each is written as a sum of two squares
// of one-FMA linear forms, x^2 + y^2:
//   k = 0:  x, y = kA0 w - u, kC0 w - u             kA0, kC0 = (11 +- sqrt 39)/8
//   k = 1:  x, y = kA1 w - u, kC1 w - u             kA1, kC1 = (5 +- sqrt 39)/8
//   k = 2:  x, y = kA0 u - w, kC0 u - w             (k = 0 mirrored)
//   k = 3:  x, y = kA3 u - w, kC3 u - w/2           kA3 = (58 - sqrt 39)/40,
//                                                   kC3 = (29 + 2 sqrt 39)/40
// (matching the coefficients: kA + kC and kA^2 + kC^2 give the cross and
// square terms).  The downwind form is kept at a quarter, 2.75 u^2 -
// 3.625 u w + 1.25 w^2 with eps / 4, so that the average of eq:SI_downwind
// is one FMA, b_3 = (b_0 + b_1 + b_2) / 4 + b_d / 4.  Likewise
// 6 tau = 1.5 t5^2 with t5 = d0 - 4 d1 + 6 d2 - 4 d3 + d4 the fifth
// difference of s (eq:GSI).  Scaling every indicator, tau and eps by the
// same factor leaves the weights unchanged.
//
// FP64 weights over a common denominator,
//   R - s_A = sum_k d_k (b_k + T) P_k (q_k - s_A) / sum_k d_k (b_k + T) P_k,
//   b_k = 6 (beta_k + eps), T = 6 tau, P_k = prod_{j != k} b_j
//   (the 1/20 of d cancels), (b_k + T) P_k = P + T P_k with P = prod_j b_j,
// algebraically identical to the normalised weights of eq:weights_unnormalized
// with one division instead of five.  These kernels run for
// 1e-70 <= eps <= 1e-40, so b_k >= 6e-70 keeps every product above 1e-276
// and nothing underflows (a smaller eps takes the general kernels); the
// products overflow only for flux values beyond about 1e37, and the
// resulting non-finite state is reported.  FP32 takes the normalised
// weights d_k (1 + T / b_k) with the hardware reciprocal instead: a product
// of four indicators would underflow at an FP32 epsilon.
// ---------------------------------------------------------------------------
template <int A, class T>
__device__ __forceinline__ T za6_diff(const T (&d)[5], const WeightCfg<T>& w) {
  static_assert(A == 2 || A == 3, "anchor s_2 or s_3");
  const T d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
  const T h4 = T(0.5) * d4;
  const T kA0 = T(2.1556247497997997757), kC0 = T(0.59437525020020022427);   // (11 +- sqrt 39)/8
  const T kA1 = T(1.4056247497997997757), kC1 = T(-0.15562474979979977573);  // (5 +- sqrt 39)/8
  const T kA3 = T(1.2938750500400400449);   // (58 - sqrt 39)/40
  const T kC3 = T(1.0372498999199199103);   // (29 + 2 sqrt 39)/40
  const T x0 = fma(kA0, d1, -d0), y0 = fma(kC0, d1, -d0);
  const T x1 = fma(kA1, d2, -d1), y1 = fma(kC1, d2, -d1);
  const T x2 = fma(kA0, d2, -d3), y2 = fma(kC0, d2, -d3);
  const T x3 = fma(kA3, d3, -d4), y3 = fma(kC3, d3, -h4);
  const T b0 = fma(x0, x0, fma(y0, y0, w.eps6));
  const T b1 = fma(x1, x1, fma(y1, y1, w.eps6));
  const T b2 = fma(x2, x2, fma(y2, y2, w.eps6));
  const T bq = fma(x3, x3, fma(y3, y3, w.eps6q));    // b_d / 4
  const T b3 = fma(T(0.25), (b0 + b1) + b2, bq);     // eq:SI_downwind
  const T t5 = fma(T(6), d2, fma(T(-4), d1 + d3, d0 + d4));
  const T tau = (T(1.5) * t5) * t5;
  T a0, a1, a2, a3;   // d_k (b_k + T) times a common factor (a1, a2: w_1/9, w_2/9 in FP64)
  if constexpr (sizeof(T) == sizeof(double)) {
    const T p01 = b0 * b1, p23 = b2 * b3;
    const T P = p01 * p23;
    a0 = fma(tau, b1 * p23, P);
    a1 = fma(tau, b0 * p23, P);
    a2 = fma(tau, p01 * b3, P);
    a3 = fma(tau, p01 * b2, P);
  } else {
    // FP32: normalised weights 1 + tau / b_k with the hardware reciprocal
    // (a product of four indicators would underflow at the FP32 epsilon)
    const T tau9 = T(9) * tau;
    a0 = fma(tau, rcp_nr(b0), T(1));
    a1 = fma(tau9, rcp_nr(b1), T(9));
    a2 = fma(tau9, rcp_nr(b2), T(9));
    a3 = fma(tau, rcp_nr(b3), T(1));
  }
  // the candidates last: fewer values live across the weights
  T t0, t1, t2, t3;
  if (A == 2) {
    t0 = fma(T(2.5), d1, -d0);
    t1 = fma(T(0.5), d1, d2);
    t2 = fma(T(-0.5), d3, d2 + d2);
    t3 = fma(T(3), d2, fma(T(-2.5), d3, d4));
  } else {
    t0 = fma(T(2.5), d1, fma(T(-3), d2, -d0));
    t1 = fma(T(0.5), d1, -(d2 + d2));
    t2 = fma(T(-0.5), d3, -d2);
    t3 = fma(T(-2.5), d3, d4);
  }
  if constexpr (sizeof(T) == sizeof(double)) {
    return div_nr(fma(a0, t0, fma(T(9), fma(a1, t1, a2 * t2), a3 * t3)), fma(T(9), a1 + a2, a0 + a3));
  } else {
    return div_nr(fma(a0, t0, fma(a1, t1, fma(a2, t2, a3 * t3))), (a0 + a1) + (a2 + a3));
  }
}

// Both Lax-Friedrichs halves of one characteristic field (eq:LF) from the
// differences dw, dg of its state and flux values between neighbouring
// stencil points: s^{+-} = g +- a w, and the negative half takes its six
// values in reverse order, whose differences are -(dg - a dw) reversed.
// Anchoring the positive half at s^+_2 and the reversed negative half at its
// fourth value s^-_2, with s^+_2 + s^-_2 = 2 g_2, gives
// F = (R^+ + R^-)/2 = g_2 + S / 6,  S = 3 (R^+ - s^+_2) + 3 (R^- - s^-_2);
// split_sum returns S.
template <class T>
__device__ __forceinline__ T split_sum(const T (&dw)[5], const T (&dg)[5], T a, const WeightCfg<T>& cfg) {
  T dp[5], dm[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    dp[k] = fma(a, dw[k], dg[k]);
    dm[4 - k] = fma(a, dw[k], -dg[k]);
  }
  return za6_diff<2>(dp, cfg) + za6_diff<3>(dm, cfg);
}

template <class T>
__device__ __forceinline__ T split_diff(const T (&dw)[5], const T (&dg)[5], T g2, T a, const WeightCfg<T>& cfg) {
  return fma(T(1.0 / 6.0), split_sum(dw, dg, a, cfg), g2);
}

// ---------------------------------------------------------------------------
// Order-2r central-upwind reconstruction for r != 3 (Section 2, Section 3 and
// Appendix A), from s = (s_0..s_{2r-1}) = 2 (f_{i-r+1}, .., f_{i+r}); returns
// twice the reconstructed flux, like za6.  Candidates on S_k (k = 0..r, S_r
// downwind), indicators as sums of squares of first differences (the printed
// quadratic forms, factored; see za_order_tables.hpp), the downwind weight's
// indicator the mean of the r upwind ones and beta_d, tau from the
// (2r-1)-th difference, Z weights (or linear / Ai / p != 1 under
// WV_GENERAL) in the direct form.  beta(2f) = 4 beta(f) and tau(2f) =
// 4 tau(f), so the epsilon is 4 eps (Ai: eps, after dividing by mu(2f)^2).
// ---------------------------------------------------------------------------
template <class T, int R, int WV>
__device__ __forceinline__ T zar(const T (&s)[2 * R], const WeightCfg<T>& w) {
  typedef OrderTables<R> Tb;
  constexpr int S = 2 * R;
  T g[S - 1];
#pragma unroll
  for (int j = 0; j < S - 1; ++j) g[j] = s[j + 1] - s[j];
  T q[R + 1];
#pragma unroll
  for (int k = 0; k <= R; ++k) {
    T acc = T(Tb::ck(k, 0)) * s[k];
#pragma unroll
    for (int j = 1; j < R; ++j) acc = fma(T(Tb::ck(k, j)), s[k + j], acc);
    q[k] = acc;
  }
  if (WV == WV_GENERAL && w.linear) {
    T acc = T(Tb::d(0)) * q[0];
#pragma unroll
    for (int k = 1; k <= R; ++k) acc = fma(T(Tb::d(k)), q[k], acc);
    return acc;
  }
  T beta[R + 1];
#pragma unroll
  for (int k = 0; k <= R; ++k) {
    T b = T(0);
#pragma unroll
    for (int l = 0; l < R - 1; ++l) {
      T t = g[k + l];
#pragma unroll
      for (int m = l + 1; m < R - 1; ++m) t = fma(T(Tb::U(k, l, m)), g[k + m], t);
      b = fma(T(Tb::lam(k, l)) * t, t, b);
    }
    beta[k] = b;
  }
  // beta[R] holds beta_d; the downwind candidate takes the mean
  T sum = beta[0];
#pragma unroll
  for (int k = 1; k <= R; ++k) sum += beta[k];
  beta[R] = sum * T(1.0 / (R + 1));
  T t5 = T(Tb::ctau(0)) * s[0];
#pragma unroll
  for (int j = 1; j < S; ++j) t5 = fma(T(Tb::ctau(j)), s[j], t5);
  T tau = t5 * t5;
  T eps = w.eps4;
  if (WV == WV_GENERAL && w.ai) {
    T mean = s[0];
#pragma unroll
    for (int j = 1; j < S; ++j) mean += s[j];
    mean *= T(1.0 / S);
    T mu = fabs(s[0] - mean);
#pragma unroll
    for (int j = 1; j < S; ++j) mu += fabs(s[j] - mean);
    mu = fma(mu, T(1.0 / S), w.mu0x2);
    const T imu2 = rcp_nr(mu * mu);
#pragma unroll
    for (int k = 0; k <= R; ++k) beta[k] *= imu2;
    tau *= imu2;
    eps = w.eps1;
  }
  T bmin = T(0);
  if (WV == WV_GENERAL && w.L == T(0)) {
    bmin = beta[0] + eps;
#pragma unroll
    for (int k = 1; k <= R; ++k) bmin = fmin(bmin, beta[k] + eps);
  }
  T num = T(0), den = T(0);
#pragma unroll
  for (int k = 0; k <= R; ++k) {
    const T a = T(Tb::d(k)) * z_alpha<T, WV>(tau, beta[k] + eps, bmin, w);
    num = fma(a, q[k], num);
    den += a;
  }
  return div_nr(num, den);
}

// Both Lax-Friedrichs halves of one characteristic field at one interface
// (eq:LF): with s^{+-}_j = g_j +- a w_j = 2 f^{+-}_j,
// F = (R(s^+_{i-r+1..i+r}) + R(s^-_{i+r..i-r+1})) / 2 where R returns twice
// the reconstruction (the Z weights at r = 3 from the differences, split_diff).
template <class T, int WV, int R = 3>
__device__ __forceinline__ T split_pair(const T (&w)[2 * R], const T (&g)[2 * R], T a, const WeightCfg<T>& cfg) {
  if constexpr (R == 3 && WV == WV_Z1) {
    T dw[5], dg[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      dw[k] = w[k + 1] - w[k];
      dg[k] = g[k + 1] - g[k];
    }
    return split_diff(dw, dg, g[2], a, cfg);
  } else {
    T p[2 * R], m[2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
      p[j] = fma(a, w[j], g[j]);
      m[j] = fma(-a, w[j], g[j]);
    }
    if constexpr (R == 3) {
      return T(0.5) * (za6<T, WV>(p[0], p[1], p[2], p[3], p[4], p[5], cfg) +
                       za6<T, WV>(m[5], m[4], m[3], m[2], m[1], m[0], cfg));
    } else {
      T mr[2 * R];
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) mr[j] = m[2 * R - 1 - j];
      return T(0.5) * (zar<T, R, WV>(p, cfg) + zar<T, R, WV>(mr, cfg));
    }
  }
}

// ---------------------------------------------------------------------------
// Per-cell records.  Everything the interface fluxes need from one cell is
// computed once per cell and sweep (point values f_j = f(Q_j), Section 2):
// the state, the physical flux and the Roe ingredients, in the sweep-normal
// frame (component 1 = normal momentum, component 2 = tangential momentum).
// Records live in LDS as structure of arrays, field f of a cell at
// rec[f * fs + offset].
//   Euler M = 4: rho, m_n, m_t, E, F1, F2, F3, 1/sqrt(rho)   (8)
//   Euler M = 3: rho, m_n, E, F1, F2, 1/sqrt(rho)            (6)
//   scalar:      u, f(u)                                    (2)
// (F0 = m_n is not stored; the Roe ingredients sqrt(rho) u and sqrt(rho) H
// of the two cells next to an interface are recomputed there from the
// state and 1/sqrt(rho), which keeps the LDS ring of the y-sweep small
// enough for three blocks per compute unit.)
// ---------------------------------------------------------------------------
template <int M> struct RecLayout;
template <> struct RecLayout<4> {
  enum { NF = 8, Q0 = 0, Q1 = 1, Q2 = 2, E = 3, F1 = 4, F2 = 5, F3 = 6, RS = 7 };
};
template <> struct RecLayout<3> {
  enum { NF = 6, Q0 = 0, Q1 = 1, Q2 = -1, E = 2, F1 = 3, F2 = -1, F3 = 4, RS = 5 };
};

// Build the record of one Euler cell from its (frame-permuted) state.
template <class T, int M>
__device__ __forceinline__ void euler_record(const double (&qd)[M], T gm1, T* rec, int fs) {
  typedef RecLayout<M> Lo;
  const T q0 = (T)qd[0], q1 = (T)qd[1], E = (T)qd[M - 1];
  const T q2 = M == 4 ? (T)qd[M == 4 ? 2 : 0] : T(0);
  T sq, hr;
  sqrt_rsq(q0, sq, hr);
  const T r = hr + hr;          // 1/sqrt(rho)
  const T ir = r * r;           // 1/rho
  const T un = q1 * ir;
  T ke;
  if (M == 4) {
    ke = fma(un, q1, (q2 * ir) * q2);
  } else {
    ke = un * q1;
  }
  const T p = gm1 * fma(T(-0.5), ke, E);
  rec[Lo::Q0 * fs] = q0;
  rec[Lo::Q1 * fs] = q1;
  rec[Lo::E * fs] = E;
  rec[Lo::F1 * fs] = fma(q1, un, p);
  rec[Lo::F3 * fs] = (E + p) * un;
  if (M == 4) {
    rec[Lo::Q2 * fs] = q2;
    rec[Lo::F2 * fs] = q2 * un;
  }
  rec[Lo::RS * fs] = r;
}

// The Roe ingredients of one record: sqrt(rho) u_n = m_n r, sqrt(rho) u_t =
// m_t r and sqrt(rho) H = (E + p) r with r = 1/sqrt(rho) and
// p = (gamma-1) (E - ((sqrt(rho) u_n)^2 + (sqrt(rho) u_t)^2)/2).
template <class T, int M>
__device__ __forceinline__ void roe_side(const T* __restrict__ rec, int fs, int o, T gm1, T& an, T& at, T& hs) {
  typedef RecLayout<M> Lo;
  const T q1 = rec[Lo::Q1 * fs + o], E = rec[Lo::E * fs + o], r = rec[Lo::RS * fs + o];
  an = q1 * r;
  T ke;
  if (M == 4) {
    at = rec[(M == 4 ? Lo::Q2 : 0) * fs + o] * r;
    ke = fma(an, an, at * at);
  } else {
    at = T(0);
    ke = an * an;
  }
  const T p = gm1 * fma(T(-0.5), ke, E);
  hs = (E + p) * r;
}

// Projection onto the characteristic fields with the left eigenvectors at the
// Roe state (factored as in euler_flux, acoustic rows scaled by 2c): of a
// state (Q0, Q1, Q2, E) or, with (Q1, F1, F2, F3) in their places, of a
// physical flux.  Linear, so it also projects differences.
template <class T, int M>
__device__ __forceinline__ void char_project(T u, T v, T q2, T k1, T b1, T Q0, T Q1, T Q2, T E, T (&W)[M]) {
  T K = fma(u, Q1, -E);
  if constexpr (M == 4) K = fma(v, Q2, K);
  const T P = fma(q2, Q0, -K);
  const T D = fma(u, Q0, -Q1);
  W[0] = fma(k1, P, D);
  W[1] = fma(-b1, P, Q0);
  if constexpr (M == 4) W[2] = fma(-v, Q0, Q2);
  W[M - 1] = fma(k1, P, -D);
}

// ---------------------------------------------------------------------------
// Characteristic-wise WENO-ZA6 (order 2R) flux of the Euler equations at one
// interface in the sweep-normal frame, from the records of its 2R-point stencil
// (value of field f at stencil point j: rec[f * fs + off[j]]).  The y-sweep
// builds its records in the permuted frame and permutes the result back; the
// two tangential fields share one eigenvalue and one LF speed, so their order
// does not change the reconstruction.
//
// Eigenvectors at the Roe average of cells i, i+1 (Section 4.2 uses the
// characteristic-wise LF splitting; Roe's average defines the state):
//   R columns (u-c, u, [u], u+c):  (1, u-c, v, H-uc), (1, u, v, q2),
//                                  (0, 0, 1, v), (1, u+c, v, H+uc)
//   L rows: A+B, Q0-2A, Q2-vQ0, A-B  with  A = (b2 Q0 - b1 K)/2,
//   B = (u Q0 - Q1)/(2c), K = u Q1 + v Q2 - E, b1 = (gamma-1)/c^2,
//   b2 = b1 q2  (the textbook left eigenvectors, factored; the rows A+B and
//   A-B are applied multiplied by 2c and the matching columns of R divided
//   by it, which leaves F = R WENO(L f) unchanged).
// ---------------------------------------------------------------------------
template <class T, int M, int WV, int R = 3>
__device__ __forceinline__ void euler_flux(const T* __restrict__ rec, int fs, const int (&off)[2 * R], T gm1,
                                           const T (&alpha)[M], const WeightCfg<T>& cfg, T (&Fh)[M]) {
  typedef RecLayout<M> Lo;
#define ZA_R(f, j) rec[(f) * fs + off[j]]
  // Roe average of the cells R-1 (= i) and R (= i+1) of the stencil:
  // u = (sqrt(rho_l) u_l + sqrt(rho_r) u_r) / (sqrt(rho_l) + sqrt(rho_r)),
  // likewise v and H, with 1/(sqrt(rho_l) + sqrt(rho_r)) = r_l r_r / (r_l + r_r)
  const T rl = ZA_R(Lo::RS, R - 1), rr = ZA_R(Lo::RS, R);
  const T iw = (rl * rr) * rcp_nr(rl + rr);
  T anl, atl, hsl, anr, atr, hsr;
  roe_side<T, M>(rec, fs, off[R - 1], gm1, anl, atl, hsl);
  roe_side<T, M>(rec, fs, off[R], gm1, anr, atr, hsr);
  const T u = (anl + anr) * iw;
  const T v = M == 4 ? (atl + atr) * iw : T(0);
  const T H = (hsl + hsr) * iw;
  const T q2 = T(0.5) * fma(u, u, v * v);
  const T c2 = gm1 * (H - q2);
  T c, hc;
  sqrt_rsq(c2, c, hc);          // c and 1/(2c)
  const T ic = hc + hc;
  const T b1 = gm1 * (ic * ic);
  const T k1 = gm1 * ic;
  // project the stencil onto the characteristic fields.  With
  // P = q2 Q0 - (u Q1 + v Q2 - E) and D = u Q0 - Q1 the left eigenvectors
  // give w_0 = (b1/2) P + D/(2c), w_3 = (b1/2) P - D/(2c), w_1 = Q0 - b1 P;
  // the acoustic fields 0 and M-1 are carried scaled by 2c, as
  // (gm1/c) P +- D, and the factor 1/(2c) is applied to the reconstructed
  // fluxes instead: one FMA per value here.  The reconstruction of a field
  // scaled by s equals s times the reconstruction of the field when the
  // indicators' epsilon is scaled by s^2 (beta and tau scale by s^2) and the
  // descaler's mu_0 by s (mu scales by s), so those two fields take
  // epsilon 4 c^2 eps and mu_0 2 c mu_0 (eq:weight_nonlinear, eq:aimu).
  if constexpr (WV == WV_Z1 && R == 3) {
    // The projection is linear, so the differences of the characteristic
    // values between neighbouring stencil points are the projections of the
    // differences of the states and fluxes between neighbouring cells, and
    // split_sum needs only those.  The FP64 kernels with the paper's Z
    // weights run only for eps <= 1e-40 (larger eps takes the general
    // kernels): there the unscaled eps, an effective eps / (4 c^2) on the
    // unscaled acoustic fields, moves a reconstruction by at most ~2e-13 of
    // the stencil's scale.  FP32 scales the acoustic fields' epsilon by
    // 4 c^2 exactly as the direct form does.  The stencil points are read one
    // at a time (a scheduling barrier per pair), which keeps the raw values
    // of two points live instead of six.
    T dW[M][5], dG[M][5], Fi[4];   // Fi: the physical flux of cell i
    T pQ0 = ZA_R(Lo::Q0, 0), pQ1 = ZA_R(Lo::Q1, 0), pE = ZA_R(Lo::E, 0);
    T pQ2 = M == 4 ? ZA_R(M == 4 ? Lo::Q2 : 0, 0) : T(0);
    T pF1 = ZA_R(Lo::F1, 0), pF3 = ZA_R(Lo::F3, 0);
    T pF2 = M == 4 ? ZA_R(M == 4 ? Lo::F2 : 0, 0) : T(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T Q0 = ZA_R(Lo::Q0, k + 1), Q1 = ZA_R(Lo::Q1, k + 1), E = ZA_R(Lo::E, k + 1);
      const T Q2 = M == 4 ? ZA_R(M == 4 ? Lo::Q2 : 0, k + 1) : T(0);
      const T F1 = ZA_R(Lo::F1, k + 1), F3 = ZA_R(Lo::F3, k + 1);
      const T F2 = M == 4 ? ZA_R(M == 4 ? Lo::F2 : 0, k + 1) : T(0);
      T w[M], g[M];
      const T dQ1 = Q1 - pQ1;
      char_project<T, M>(u, v, q2, k1, b1, Q0 - pQ0, dQ1, Q2 - pQ2, E - pE, w);
      char_project<T, M>(u, v, q2, k1, b1, dQ1, F1 - pF1, F2 - pF2, F3 - pF3, g);
#pragma unroll
      for (int f = 0; f < M; ++f) {
        dW[f][k] = w[f];
        dG[f][k] = g[f];
      }
      if (k + 1 == R - 1) { Fi[0] = Q1; Fi[1] = F1; Fi[2] = F2; Fi[3] = F3; }
      pQ0 = Q0; pQ1 = Q1; pQ2 = Q2; pE = E; pF1 = F1; pF2 = F2; pF3 = F3;
      __builtin_amdgcn_sched_barrier(0);
    }
    WeightCfg<T> cfg_ac = cfg;
    if constexpr (sizeof(T) == sizeof(float)) {
      cfg_ac.eps6 = cfg.eps6 * (T(4) * c2);
      cfg_ac.eps6q = cfg.eps6q * (T(4) * c2);
    }
    T S[M];
    S[0] = split_sum(dW[0], dG[0], alpha[0], cfg_ac);
    S[M - 1] = split_sum(dW[M - 1], dG[M - 1], alpha[M - 1], cfg_ac);
#pragma unroll
    for (int f = 1; f < M - 1; ++f) S[f] = split_sum(dW[f], dG[f], alpha[f], cfg);
    // F = R (g_i + S / 6) with g_i = L F(Q_i), the projected flux of cell i,
    // and R L = I: F = F(Q_i) + R S / 6, the back-projection below with the
    // factor 1/6 folded into its constants and the acoustic fields unscaled
    // by 1/(2c) as in the direct form.
    const T k6 = T(1.0 / 6.0);
    const T s03 = (S[0] + S[M - 1]) * (hc * k6);
    const T d30 = T(0.5 / 6.0) * (S[M - 1] - S[0]);
    const T sum = fma(k6, S[1], s03);
    Fh[0] = Fi[0] + sum;
    Fh[1] = Fi[1] + fma(u, sum, d30);
    if constexpr (M == 4) {
      const T s2 = k6 * S[2];
      Fh[2] = Fi[2] + fma(v, sum, s2);
      Fh[3] = Fi[3] + fma(H, s03, fma(u, d30, fma(q2 * k6, S[1], v * s2)));
    } else {
      Fh[2] = Fi[3] + fma(H, s03, fma(u, d30, (q2 * k6) * S[1]));
    }
  } else {
    T gh[M];
    T W[M][2 * R], G[M][2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
      const T Q0 = ZA_R(Lo::Q0, j), Q1 = ZA_R(Lo::Q1, j), E = ZA_R(Lo::E, j);
      const T Q2 = M == 4 ? ZA_R(M == 4 ? Lo::Q2 : 0, j) : T(0);
      const T F1 = ZA_R(Lo::F1, j), F3 = ZA_R(Lo::F3, j);
      const T F2 = M == 4 ? ZA_R(M == 4 ? Lo::F2 : 0, j) : T(0);
      {
        T K = fma(u, Q1, -E);
        if (M == 4) K = fma(v, Q2, K);
        const T P = fma(q2, Q0, -K);
        const T D = fma(u, Q0, -Q1);
        W[0][j] = fma(k1, P, D);
        W[1][j] = fma(-b1, P, Q0);
        if (M == 4) W[2][j] = fma(-v, Q0, Q2);
        W[M - 1][j] = fma(k1, P, -D);
      }
      {
        // physical flux (F0 = Q1, F1, [F2], F3)
        T K = fma(u, F1, -F3);
        if (M == 4) K = fma(v, F2, K);
        const T P = fma(q2, Q1, -K);
        const T D = fma(u, Q1, -F1);
        G[0][j] = fma(k1, P, D);
        G[1][j] = fma(-b1, P, Q1);
        if (M == 4) G[2][j] = fma(-v, Q1, F2);
        G[M - 1][j] = fma(k1, P, -D);
      }
    }
    // The FP64 kernels with the paper's Z weights run only for eps <= 1e-40
    // (larger eps takes the general kernels): there the unscaled eps, an
    // effective eps / (4 c^2) on the unscaled fields, moves a reconstruction
    // by at most ~2e-13 of the stencil's scale, and the kernels keep the
    // registers the per-interface eps would take.
    constexpr bool scale_eps = !(WV == WV_Z1 && sizeof(T) == sizeof(double));
    WeightCfg<T> cfg_ac = cfg;
    if (scale_eps) {
      if (WV == WV_GENERAL && cfg.ai) {
        cfg_ac.mu0x2 = cfg.mu0x2 * (c + c);
      } else {
        const T s2 = T(4) * c2;
        cfg_ac.eps16 = cfg.eps16 * s2;
        cfg_ac.eps4 = cfg.eps4 * s2;
      }
    }
    // the two acoustic fields first, so that their epsilon dies early
    gh[0] = split_pair<T, WV, R>(W[0], G[0], alpha[0], cfg_ac);
    gh[M - 1] = split_pair<T, WV, R>(W[M - 1], G[M - 1], alpha[M - 1], cfg_ac);
#pragma unroll
    for (int s = 1; s < M - 1; ++s) gh[s] = split_pair<T, WV, R>(W[s], G[s], alpha[s], cfg);
    // back-projection F = R g, the acoustic fluxes unscaled by 1/(2c):
    // gh_0 + gh_3 = (gh'_0 + gh'_3)/(2c), c (gh_3 - gh_0) = (gh'_3 - gh'_0)/2
    const T s03 = (gh[0] + gh[M - 1]) * (T(0.5) * ic);
    const T d30 = T(0.5) * (gh[M - 1] - gh[0]);
    const T sum = s03 + gh[1];
    Fh[0] = sum;
    Fh[1] = fma(u, sum, d30);
    if (M == 4) {
      Fh[2] = fma(v, sum, gh[2]);
      Fh[3] = fma(H, s03, fma(u, d30, fma(q2, gh[1], v * gh[2])));
    } else {
      Fh[2] = fma(H, s03, fma(u, d30, q2 * gh[1]));
    }
  }
#undef ZA_R
}

}  // namespace za
