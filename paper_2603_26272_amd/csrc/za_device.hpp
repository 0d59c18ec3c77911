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
#include <stdint.h>

namespace za {

// ---------------------------------------------------------------------------
// Parameters of the nonlinear weights (eq:weight_nonlinear, eq:aimu).
// ---------------------------------------------------------------------------
template <class T>
struct WeightCfg {
  T eps;      // sensitivity epsilon
  T mu0;      // mu_0 of the affine-invariant descaler
  T p;        // power parameter (1 on the fast path)
  int ai;     // 1: affine-invariant descaler
  int linear; // 1: omega = d
};

template <class T> __device__ __forceinline__ T rcp_fast(T x);
template <> __device__ __forceinline__ float rcp_fast<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp_fast<double>(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// One WENO-ZA6 reconstruction of h at x_{i+1/2} from v0..v5 = f_{i-2..i+3}
// (Section 3: r = 3).  The negative split flux calls this with the six
// values in reverse order (mirror symmetry about x_{i+1/2}, Section 2).
//
//  candidates  q_k = <c_k, f_k>, c_k = (2,-7,11)/6, (-1,5,2)/6, (2,5,-1)/6,
//              (11,-7,2)/6                         (eq:subflux_S6_coeffs)
//  indicators  beta_k = (13/12) D2_k^2 + (1/4) D1_k^2, the Jiang-Shu form of
//              eq:SI for quadratics (D2 the second difference, D1 twice the
//              slope of p_k at x_i); k = 3 is the downwind beta_d measured on
//              I_i.  This sum of squares equals the printed quadratic forms
//              <f_k, B_k f_k> (eq:SI_S6) exactly and is never negative.
//  downwind    beta_3 = (beta_0 + beta_1 + beta_2 + beta_d)/4 (eq:SI_downwind)
//  global      tau = <c_tau, f>^2, c_tau = (-1,5,-10,10,-5,1)   (eq:GSI)
//  weights     alpha_k = d_k (1 + tau/(beta_k + eps mu^2)), d = (1,9,9,1)/20,
//              omega_k = alpha_k / sum alpha  (eq:weights_unnormalized with
//              L = q = 1, p = 1, eq:weights_general)
//
// FP64, p = 1: the weights are evaluated over a common denominator,
//   f = sum_k d_k (b_k + tau) P_k q_k / sum_k d_k (b_k + tau) P_k,
//   b_k = beta_k + eps, P_k = prod_{j != k} b_j,
// which is algebraically identical and needs one division instead of five.
// b_k >= eps = 1e-40 keeps every product above 1e-161 (no underflow in FP64);
// with the Ai descaler the indicators are first divided by mu^2, which
// leaves Gamma_k unchanged and restores b_k >= eps.  FP32 keeps the direct
// form (products of three indicators would underflow at eps = 1e-20) with
// hardware reciprocals.
// ---------------------------------------------------------------------------
template <class T, bool GENERIC_P>
__device__ __forceinline__ T za6(T v0, T v1, T v2, T v3, T v4, T v5, const WeightCfg<T>& w) {
  const T sixth = T(1) / T(6);
  T q0 = (T(2) * v0 - T(7) * v1 + T(11) * v2) * sixth;
  T q1 = (-v1 + T(5) * v2 + T(2) * v3) * sixth;
  T q2 = (T(2) * v2 + T(5) * v3 - v4) * sixth;
  T q3 = (T(11) * v3 - T(7) * v4 + T(2) * v5) * sixth;
  if (w.linear) {
    return (q0 + T(9) * q1 + T(9) * q2 + q3) * (T(1) / T(20));
  }
  const T c13 = T(13) / T(12), c14 = T(0.25);
  T a = v0 - T(2) * v1 + v2, b = v0 - T(4) * v1 + T(3) * v2;
  T be0 = c13 * a * a + c14 * b * b;
  a = v1 - T(2) * v2 + v3; b = v1 - v3;
  T be1 = c13 * a * a + c14 * b * b;
  a = v2 - T(2) * v3 + v4; b = T(3) * v2 - T(4) * v3 + v4;
  T be2 = c13 * a * a + c14 * b * b;
  a = v3 - T(2) * v4 + v5; b = T(-5) * v3 + T(8) * v4 - T(3) * v5;
  T bed = c13 * a * a + c14 * b * b;
  T be3 = T(0.25) * (be0 + be1 + be2 + bed);
  T t5 = (v5 - v0) + T(5) * (v1 - v4) + T(10) * (v3 - v2);
  T tau = t5 * t5;
  T eps = w.eps;
  if (w.ai) {
    T mean = (v0 + v1 + v2 + v3 + v4 + v5) * sixth;
    T mu = (fabs(v0 - mean) + fabs(v1 - mean) + fabs(v2 - mean) + fabs(v3 - mean) +
            fabs(v4 - mean) + fabs(v5 - mean)) * sixth + w.mu0;
    T imu2 = T(1) / (mu * mu);
    be0 *= imu2; be1 *= imu2; be2 *= imu2; be3 *= imu2; tau *= imu2;
  }
  T b0 = be0 + eps, b1 = be1 + eps, b2 = be2 + eps, b3 = be3 + eps;
  if (GENERIC_P || sizeof(T) == 4) {
    T g0 = tau * rcp_fast<T>(b0), g1 = tau * rcp_fast<T>(b1);
    T g2 = tau * rcp_fast<T>(b2), g3 = tau * rcp_fast<T>(b3);
    if (GENERIC_P) {
      g0 = pow(g0, w.p); g1 = pow(g1, w.p); g2 = pow(g2, w.p); g3 = pow(g3, w.p);
    }
    T a0 = T(1) + g0, a1 = T(9) * (T(1) + g1), a2 = T(9) * (T(1) + g2), a3 = T(1) + g3;
    return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) * rcp_fast<T>(a0 + a1 + a2 + a3);
  } else {
    T p01 = b0 * b1, p23 = b2 * b3;
    T e0 = (b0 + tau) * (b1 * p23);
    T e1 = T(9) * (b1 + tau) * (b0 * p23);
    T e2 = T(9) * (b2 + tau) * (p01 * b3);
    T e3 = (b3 + tau) * (p01 * b2);
    return (e0 * q0 + e1 * q1 + e2 * q2 + e3 * q3) / (e0 + e1 + e2 + e3);
  }
}

// Both Lax-Friedrichs halves of one field at one interface (eq:LF):
// g^{+-}_j = (g_j +- a w_j)/2; F = R^+(g^+_{i-2..i+3}) + R^+(g^-_{i+3..i-2}).
template <class T, bool GP>
__device__ __forceinline__ T split_pair(const T (&w)[6], const T (&g)[6], T a, const WeightCfg<T>& cfg) {
  T p[6], m[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    p[j] = T(0.5) * (g[j] + a * w[j]);
    m[j] = T(0.5) * (g[j] - a * w[j]);
  }
  return za6<T, GP>(p[0], p[1], p[2], p[3], p[4], p[5], cfg) +
         za6<T, GP>(m[5], m[4], m[3], m[2], m[1], m[0], cfg);
}

// ---------------------------------------------------------------------------
// Characteristic-wise WENO-ZA6 flux of the Euler equations at one interface,
// in the sweep-normal frame: component 1 of the state is the normal momentum
// and (for M = 4) component 2 the tangential one.  The y-sweep permutes its
// state into this frame and the result back; the two tangential-velocity
// fields share one eigenvalue and one LF speed, so the reconstruction does
// not depend on their order.
//
// Eigenvectors at the Roe average of cells i, i+1 (Section 4.2 uses the
// characteristic-wise LF splitting; Roe's average defines the state):
//   R columns (u-c, u, [u], u+c):  (1, u-c, v, H-uc), (1, u, v, q2),
//                                  (0, 0, 1, v), (1, u+c, v, H+uc)
//   L rows: A+B, Q0-2A, Q2-vQ0, A-B  with  A = (b2 Q0 - b1 K)/2,
//   B = (u Q0 - Q1)/(2c), K = u Q1 + v Q2 - E, b1 = (gamma-1)/c^2,
//   b2 = b1 q2  (the textbook left eigenvectors, factored).
// ---------------------------------------------------------------------------
template <class T, int M, bool GP>
__device__ __forceinline__ void euler_flux(const double (&qs)[6][M], T gm1, const T (&alpha)[M],
                                           const WeightCfg<T>& cfg, T (&Fh)[M]) {
  // primitive variables and physical flux of the six cells (point values)
  T Q[6][M], F[6][M], un[6], ut[6], pr[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
#pragma unroll
    for (int c = 0; c < M; ++c) Q[j][c] = (T)qs[j][c];
    T ir = T(1) / Q[j][0];
    un[j] = Q[j][1] * ir;
    T ke;
    if (M == 4) {
      ut[j] = Q[j][2] * ir;
      ke = un[j] * Q[j][1] + ut[j] * Q[j][2];
    } else {
      ut[j] = T(0);
      ke = un[j] * Q[j][1];
    }
    pr[j] = gm1 * (Q[j][M - 1] - T(0.5) * ke);
    F[j][0] = Q[j][1];
    F[j][1] = Q[j][1] * un[j] + pr[j];
    if (M == 4) F[j][2] = Q[j][2] * un[j];
    F[j][M - 1] = (Q[j][M - 1] + pr[j]) * un[j];
  }
  // Roe average of cells 2 (= i) and 3 (= i+1)
  T sl = sqrt(Q[2][0]), sr = sqrt(Q[3][0]);
  T iw = T(1) / (sl + sr);
  T wl = sl * iw, wr = sr * iw;
  T Hl = (Q[2][M - 1] + pr[2]) / Q[2][0], Hr = (Q[3][M - 1] + pr[3]) / Q[3][0];
  T u = wl * un[2] + wr * un[3];
  T v = (M == 4) ? wl * ut[2] + wr * ut[3] : T(0);
  T H = wl * Hl + wr * Hr;
  T q2 = T(0.5) * (u * u + v * v);
  T c2 = gm1 * (H - q2);
  T c = sqrt(c2);
  T ic = T(1) / c;
  T b1 = gm1 * (ic * ic);
  T b2 = b1 * q2;
  T hic = T(0.5) * ic;
  // project the stencil onto the characteristic fields
  T W[M][6], G[M][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    {
      T K = u * Q[j][1] - Q[j][M - 1];
      if (M == 4) K += v * Q[j][2];
      T A = T(0.5) * (b2 * Q[j][0] - b1 * K);
      T B = hic * (u * Q[j][0] - Q[j][1]);
      W[0][j] = A + B;
      W[1][j] = Q[j][0] - T(2) * A;
      if (M == 4) W[2][j] = Q[j][2] - v * Q[j][0];
      W[M - 1][j] = A - B;
    }
    {
      T K = u * F[j][1] - F[j][M - 1];
      if (M == 4) K += v * F[j][2];
      T A = T(0.5) * (b2 * F[j][0] - b1 * K);
      T B = hic * (u * F[j][0] - F[j][1]);
      G[0][j] = A + B;
      G[1][j] = F[j][0] - T(2) * A;
      if (M == 4) G[2][j] = F[j][2] - v * F[j][0];
      G[M - 1][j] = A - B;
    }
  }
  T gh[M];
#pragma unroll
  for (int s = 0; s < M; ++s) gh[s] = split_pair<T, GP>(W[s], G[s], alpha[s], cfg);
  // back-projection F = R g
  T s03 = gh[0] + gh[M - 1], d30 = gh[M - 1] - gh[0];
  T sum = s03 + gh[1];
  Fh[0] = sum;
  Fh[1] = u * sum + c * d30;
  if (M == 4) {
    Fh[2] = v * sum + gh[2];
    Fh[3] = H * s03 + (u * c) * d30 + q2 * gh[1] + v * gh[2];
  } else {
    Fh[2] = H * s03 + (u * c) * d30 + q2 * gh[1];
  }
}

}  // namespace za
