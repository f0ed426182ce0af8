// adjoint.h -- hand-written reverse-mode (vector-Jacobian) arithmetic of the
// per-cell and per-face operations in device.h: cons->prim, prim->cons,
// WENO5-JS and HLLC.  Each function recomputes the forward quantities it needs
// from its inputs and accumulates cotangents (+=) into the input cotangents.
// Branches (min/max of wave speeds, HLLC regions) follow the forward branch;
// ties go to the first argument exactly as in the forward code.
#pragma once

#include "device.h"

namespace mfc {

// cons->prim adjoint: given wbar (cotangent of alpha_i rho_i, u_d, p, alpha_i)
// at the state U, accumulate Ubar.  Forward: rho = sum alpha_i rho_i,
// u = m/rho, p = (E - |m|^2/(2 rho) - Pi)/Gamma, Gamma/Pi linear in alpha.
template <int NF, int D>
__host__ __device__ __forceinline__ void cons_to_prim_vjp(const Params& pm, const double* U, const double* wbar,
                                                          double* Ubar) {
  using R = Rows<NF, D>;
  double rho = U[0];
  if constexpr (NF == 2) rho = U[0] + U[1];
  const double rinv = fast_rcp(rho);
  double u[D];
  double usq = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[d] = U[R::MOM + d] * rinv;
    usq += u[d] * u[d];
  }
  double Gam, Pi;
  if constexpr (NF == 2)
    mixture<NF, double>(pm, U[R::ALPHA], U[R::ALPHA + 1], Gam, Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, Gam, Pi);
  const double gi = fast_rcp(Gam);
  const double p = (U[R::E] - 0.5 * rho * usq - Pi) * gi;
  const double pb = wbar[R::E];
  Ubar[R::E] += pb * gi;
  const double keb = -pb * gi;   // d p / d ke
  const double Pib = -pb * gi;   // d p / d Pi
  const double Gamb = -pb * p * gi;
  double rhob = keb * (-0.5 * usq);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double ub = wbar[R::MOM + d];
    Ubar[R::MOM + d] += ub * rinv + keb * u[d];
    rhob -= ub * u[d] * rinv;
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) Ubar[i] += wbar[i] + rhob;
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) Ubar[R::ALPHA + j] += wbar[R::ALPHA + j] + Gamb * pm.G[j] + Pib * pm.P[j];
  }
}

// prim->cons adjoint: given qbar at the primitive state W, accumulate Wbar.
// Forward: m = rho u, E = Gamma p + Pi + rho |u|^2 / 2.
template <int NF, int D>
__host__ __device__ __forceinline__ void prim_to_cons_vjp(const Params& pm, const double* W, const double* qbar,
                                                          double* Wbar) {
  using R = Rows<NF, D>;
  double rho = W[0];
  if constexpr (NF == 2) rho = W[0] + W[1];
  double usq = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) usq += W[R::MOM + d] * W[R::MOM + d];
  double Gam, Pi;
  if constexpr (NF == 2)
    mixture<NF, double>(pm, W[R::ALPHA], W[R::ALPHA + 1], Gam, Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, Gam, Pi);
  const double Eb = qbar[R::E];
  double rhob = Eb * 0.5 * usq;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double mb = qbar[R::MOM + d];
    const double u = W[R::MOM + d];
    Wbar[R::MOM + d] += mb * rho + Eb * rho * u;
    rhob += mb * u;
  }
  Wbar[R::E] += Eb * Gam;
#pragma unroll
  for (int i = 0; i < NF; ++i) Wbar[i] += qbar[i] + rhob;
  if constexpr (NF == 2) {
    const double p = W[R::E];
#pragma unroll
    for (int j = 0; j < 2; ++j) Wbar[R::ALPHA + j] += qbar[R::ALPHA + j] + (Eb * p) * pm.G[j] + Eb * pm.P[j];
  }
}

// Adjoint of the left-biased WENO5-JS value at i+1/2 from f = (a, b, c, d, e),
// in the difference form of the forward: with D0..D3 the consecutive
// differences, y = c + sum_k w_k l_k / 6, w_k = d_k s_k^-2 / sum_j d_j s_j^-2,
// s_k = 4 (eps + beta_k) (a common factor the weights ignore), and
// l_0 = 5D1 - 2D0, l_1 = D1 + 2D2, l_2 = 4D2 - D3 six times the candidate
// corrections.  One refined reciprocal of N * s0 s1 s2 with
// N = sum_k d_k prod_{j != k} s_j^2 gives both 1/N (the weights) and
// 1/(s0 s1 s2) (the indicator derivatives dy/ds_k = -2 w_k (l_k/6 - (y - c))/s_k).
// Accumulates g[0..4].
__host__ __device__ __forceinline__ void weno_left_vjp(double a, double b, double c, double d, double e,
                                                       double eps, double gy, double* g) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;   // prod_{j != k} s_j
  const double n0 = 0.1 * (m0 * m0), n1 = 0.6 * (m1 * m1), n2 = 0.3 * (m2 * m2);
  const double N = n0 + n1 + n2;
  const double P = s0 * m0;
  const double inv = fast_rcp(N * P);
  const double rN = P * inv;    // 1/N
  const double rP = N * inv;    // 1/(s0 s1 s2)
  const double w0 = n0 * rN, w1 = n1 * rN, w2 = n2 * rN;
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double k6 = 1.0 / 6.0;
  const double dy = (w0 * l0 + w1 * l1 + w2 * l2) * k6;
  // cotangents of l_k and s_k
  const double gk = gy * k6;
  const double gl0 = gk * w0, gl1 = gk * w1, gl2 = gk * w2;
  const double g2 = -2.0 * gy * rP;
  const double gs0 = g2 * w0 * (l0 * k6 - dy) * m0;
  const double gs1 = g2 * w1 * (l1 * k6 - dy) * m1;
  const double gs2 = g2 * w2 * (l2 * k6 - dy) * m2;
  const double gu0 = gs0 * (26.0 / 3.0) * u0, gv0 = gs0 * 2.0 * v0;
  const double gu1 = gs1 * (26.0 / 3.0) * u1, gv1 = gs1 * 2.0 * v1;
  const double gu2 = gs2 * (26.0 / 3.0) * u2, gv2 = gs2 * 2.0 * v2;
  // back to the differences, then to the five values
  const double gD0 = -2.0 * gl0 - gu0 - gv0;
  const double gD1 = 5.0 * gl0 + gl1 + gu0 + 3.0 * gv0 - gu1 + gv1;
  const double gD2 = 2.0 * gl1 + 4.0 * gl2 + gu1 + gv1 - gu2 - 3.0 * gv2;
  const double gD3 = -gl2 + gu2 + gv2;
  g[0] -= gD0;
  g[1] += gD0 - gD1;
  g[2] += gy + gD1 - gD2;
  g[3] += gD2 - gD3;
  g[4] += gD3;
}

// Adjoint of the left-biased WENO5-Z value (Sec. 4.2.2) in the same difference
// form: with s_k = 4 (eps + beta_k) and tau = |s_0 - s_2|, the weights are
// a_k = d_k (s_k + tau)/s_k and y = c + sum_k w_k l_k/6, w_k = a_k/A, A = sum a_k.
// Cotangents: of a_k, G_k = gy (l_k/6 - (y - c))/A; of s_k through a_k,
// -G_k d_k tau/s_k^2; of tau, sum_k G_k d_k/s_k, which reaches s_0 and s_2 with
// the sign of s_0 - s_2 (none at a tie).  One refined reciprocal of
// Z s_0 s_1 s_2 (Z = A s_0 s_1 s_2) gives 1/Z, 1/A and every 1/s_k.
// Accumulates g[0..4].
__host__ __device__ __forceinline__ void weno_z_left_vjp(double a, double b, double c, double d, double e,
                                                         double eps, double gy, double* g) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double tau = fabs(s0 - s2);
  const double m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;   // prod_{j != k} s_j
  const double P = s0 * m0;
  const double z0 = 0.1 * ((s0 + tau) * m0), z1 = 0.6 * ((s1 + tau) * m1), z2 = 0.3 * ((s2 + tau) * m2);
  const double Z = z0 + z1 + z2;
  const double inv = fast_rcp(Z * P);
  const double rZ = P * inv;    // 1/Z
  const double rA = P * rZ;     // 1/A
  const double rP = Z * inv;    // 1/(s0 s1 s2)
  const double w0 = z0 * rZ, w1 = z1 * rZ, w2 = z2 * rZ;
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double k6 = 1.0 / 6.0;
  const double dy = (w0 * l0 + w1 * l1 + w2 * l2) * k6;
  // cotangents of l_k, of the weights a_k, of tau and of s_k
  const double gk = gy * k6;
  const double gl0 = gk * w0, gl1 = gk * w1, gl2 = gk * w2;
  const double G0 = gy * (l0 * k6 - dy) * rA, G1 = gy * (l1 * k6 - dy) * rA, G2 = gy * (l2 * k6 - dy) * rA;
  const double rs0 = m0 * rP, rs1 = m1 * rP, rs2 = m2 * rP;
  const double gtau = 0.1 * G0 * rs0 + 0.6 * G1 * rs1 + 0.3 * G2 * rs2;
  const double sg = (s0 > s2) ? 1.0 : ((s0 < s2) ? -1.0 : 0.0);
  const double gs0 = -0.1 * G0 * tau * (rs0 * rs0) + sg * gtau;
  const double gs1 = -0.6 * G1 * tau * (rs1 * rs1);
  const double gs2 = -0.3 * G2 * tau * (rs2 * rs2) - sg * gtau;
  const double gu0 = gs0 * (26.0 / 3.0) * u0, gv0 = gs0 * 2.0 * v0;
  const double gu1 = gs1 * (26.0 / 3.0) * u1, gv1 = gs1 * 2.0 * v1;
  const double gu2 = gs2 * (26.0 / 3.0) * u2, gv2 = gs2 * 2.0 * v2;
  // back to the differences, then to the five values
  const double gD0 = -2.0 * gl0 - gu0 - gv0;
  const double gD1 = 5.0 * gl0 + gl1 + gu0 + 3.0 * gv0 - gu1 + gv1;
  const double gD2 = 2.0 * gl1 + 4.0 * gl2 + gu1 + gv1 - gu2 - 3.0 * gv2;
  const double gD3 = -gl2 + gu2 + gv2;
  g[0] -= gD0;
  g[1] += gD0 - gD1;
  g[2] += gy + gD1 - gD2;
  g[3] += gD2 - gD3;
  g[4] += gD3;
}

// Adjoint of the left-biased WENO5-M value (mapped JS weights, Sec. 3.2.1).
// Forward: JS weights w_k = n_k/N (n_k = d_k prod_{j != k} s_j^2), mapped
// h_k = g_k(w_k) = num_k/den_k, weights W_k = h_k / sum h, y = c + sum W_k l_k/6.
// Cotangents: of h_k, gy (l_k/6 - (y - c)) / sum h; of w_k, that times
// g_k'(w_k) = (num_k' den_k - num_k (1 - 2 d_k)) / den_k^2 with num_k' =
// d_k + d_k^2 - 6 d_k w_k + 3 w_k^2; of s_k, -2 w_k (wbar_k - sum_j wbar_j w_j)/s_k
// (the JS normalization), then as in weno_left_vjp.  Accumulates g[0..4].
__host__ __device__ __forceinline__ void weno_m_left_vjp(double a, double b, double c, double d, double e,
                                                         double eps, double gy, double* g) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;   // prod_{j != k} s_j
  const double n0 = 0.1 * (m0 * m0), n1 = 0.6 * (m1 * m1), n2 = 0.3 * (m2 * m2);
  const double N = n0 + n1 + n2;
  const double P = s0 * m0;
  const double inv = fast_rcp(N * P);
  const double rN = P * inv;    // 1/N
  const double rP = N * inv;    // 1/(s0 s1 s2)
  const double w0 = n0 * rN, w1 = n1 * rN, w2 = n2 * rN;
  double num0, den0, num1, den1, num2, den2;
  weno_m_map(w0, 0.1, num0, den0);
  weno_m_map(w1, 0.6, num1, den1);
  weno_m_map(w2, 0.3, num2, den2);
  const double c0 = den1 * den2, c1 = den0 * den2, c2 = den0 * den1;   // prod_{j != k} den_j
  const double E0 = num0 * c0, E1 = num1 * c1, E2 = num2 * c2;
  const double H = E0 + E1 + E2;
  const double Q = den0 * c0;
  const double inv2 = fast_rcp(H * Q);
  const double rH = Q * inv2;   // 1/H
  const double rQ = H * inv2;   // 1/(den0 den1 den2)
  const double W0 = E0 * rH, W1 = E1 * rH, W2 = E2 * rH;
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double k6 = 1.0 / 6.0;
  const double dy = (W0 * l0 + W1 * l1 + W2 * l2) * k6;
  const double gk = gy * k6;
  const double gl0 = gk * W0, gl1 = gk * W1, gl2 = gk * W2;
  // cotangents of the mapped values h_k = num_k/den_k: 1/sum h = Q/H
  const double gh = gy * (Q * rH);
  const double gh0 = gh * (l0 * k6 - dy), gh1 = gh * (l1 * k6 - dy), gh2 = gh * (l2 * k6 - dy);
  // of the JS weights through the map (1/den_k = c_k / Q)
  const double id0 = c0 * rQ, id1 = c1 * rQ, id2 = c2 * rQ;
  const double dn0 = (0.1 + 0.01) + w0 * (3.0 * w0 - 0.6);
  const double dn1 = (0.6 + 0.36) + w1 * (3.0 * w1 - 3.6);
  const double dn2 = (0.3 + 0.09) + w2 * (3.0 * w2 - 1.8);
  const double gw0 = gh0 * ((dn0 - num0 * (0.8 * id0)) * id0);
  const double gw1 = gh1 * ((dn1 - num1 * (-0.2 * id1)) * id1);
  const double gw2 = gh2 * ((dn2 - num2 * (0.4 * id2)) * id2);
  const double cw = gw0 * w0 + gw1 * w1 + gw2 * w2;
  // of s_k through the JS normalization (1/s_k = m_k / (s0 s1 s2))
  const double gs0 = -2.0 * w0 * (gw0 - cw) * (m0 * rP);
  const double gs1 = -2.0 * w1 * (gw1 - cw) * (m1 * rP);
  const double gs2 = -2.0 * w2 * (gw2 - cw) * (m2 * rP);
  const double gu0 = gs0 * (26.0 / 3.0) * u0, gv0 = gs0 * 2.0 * v0;
  const double gu1 = gs1 * (26.0 / 3.0) * u1, gv1 = gs1 * 2.0 * v1;
  const double gu2 = gs2 * (26.0 / 3.0) * u2, gv2 = gs2 * 2.0 * v2;
  const double gD0 = -2.0 * gl0 - gu0 - gv0;
  const double gD1 = 5.0 * gl0 + gl1 + gu0 + 3.0 * gv0 - gu1 + gv1;
  const double gD2 = 2.0 * gl1 + 4.0 * gl2 + gu1 + gv1 - gu2 - 3.0 * gv2;
  const double gD3 = -gl2 + gu2 + gv2;
  g[0] -= gD0;
  g[1] += gD0 - gD1;
  g[2] += gy + gD1 - gD2;
  g[3] += gD2 - gD3;
  g[4] += gD3;
}

// Adjoint of the left-biased TENO5 value (Sec. 4.2.2): the kept set is decided
// exactly as in the forward reconstruction and the weights are then constant,
// so y = c + sum_k w_k l_k / 6 with w_k = d_k delta_k / sum d delta is linear
// in the differences.  Accumulates g[0..4].
__host__ __device__ __forceinline__ void teno_left_vjp(double a, double b, double c, double d, double e,
                                                       double eps, double gy, double* g) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double tau = fabs(s0 - s2);
  const double m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;
  const double rP = fast_rcp(s0 * m0);
  const double x0 = 1.0 + tau * (m0 * rP), x1 = 1.0 + tau * (m1 * rP), x2 = 1.0 + tau * (m2 * rP);
  const double g0 = 0.1 * ((x0 * x0) * (x0 * x0) * (x0 * x0));
  const double g1 = 0.6 * ((x1 * x1) * (x1 * x1) * (x1 * x1));
  const double g2 = 0.3 * ((x2 * x2) * (x2 * x2) * (x2 * x2));
  const double cut = kTenoCt * (g0 + g1 + g2);
  const double w0 = g0 >= cut ? 0.1 : 0.0, w1 = g1 >= cut ? 0.6 : 0.0, w2 = g2 >= cut ? 0.3 : 0.0;
  const double gk = gy * fast_rcp(6.0 * (w0 + w1 + w2));
  const double gl0 = gk * w0, gl1 = gk * w1, gl2 = gk * w2;
  // l_0 = 5D1 - 2D0, l_1 = D1 + 2D2, l_2 = 4D2 - D3
  const double gD0 = -2.0 * gl0;
  const double gD1 = 5.0 * gl0 + gl1;
  const double gD2 = 2.0 * gl1 + 4.0 * gl2;
  const double gD3 = -gl2;
  g[0] -= gD0;
  g[1] += gD0 - gD1;
  g[2] += gy + gD1 - gD2;
  g[3] += gD2 - gD3;
  g[4] += gD3;
}

// Adjoint of one reconstruction centre: gL is the cotangent of the left-biased
// value at i+1/2, gR of the right-biased value at i-1/2 (the mirror image).
__host__ __device__ __forceinline__ void weno5_js_vjp(const double* f, double eps, double gL, double gR, double* g) {
  weno_left_vjp(f[0], f[1], f[2], f[3], f[4], eps, gL, g);
  double gr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  weno_left_vjp(f[4], f[3], f[2], f[1], f[0], eps, gR, gr);
  g[0] += gr[4];
  g[1] += gr[3];
  g[2] += gr[2];
  g[3] += gr[1];
  g[4] += gr[0];
}

// ---------------------------------------------------------------------------
// Adjoint of the non-uniform WENO5-JS of one centre (weno5_nu): with
// cotangents gR of the value at the right face and gL of the value at the
// left face, accumulates g[0..4] of the five cell values.  Forward: per
// candidate r, m0' = mu0 (D_r, D_{r+1}), m1, m2 linear in the two differences,
// values f_2 + m0' + m2/4 +- m1/2, indicator beta_r = m1^2 + (13/3) m2^2,
// weights d_r/(eps + beta_r)^2 normalized per face.  Reverse: the candidate
// cotangents are g omega_r, and beta_r collects -2/(eps + beta_r) times
// g omega_r (q_r - (y - f_2)) from each face.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void weno_nu_vjp(double a, double b, double c, double d, double e, double eps,
                                            const double* cf, long long st, double gR, double gL, double* g) {
  const double D[4] = {b - a, c - b, d - c, e - d};
  double qr[3], ql[3], beta[3], m1[3], m2[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double da = D[r], db = D[r + 1];
    const double mu0 = cf[(NU_MU0 + 2 * r) * st] * da + cf[(NU_MU0 + 2 * r + 1) * st] * db;
    m1[r] = cf[(NU_M1 + 2 * r) * st] * da + cf[(NU_M1 + 2 * r + 1) * st] * db;
    m2[r] = cf[(NU_M2 + 2 * r) * st] * da + cf[(NU_M2 + 2 * r + 1) * st] * db;
    const double even = mu0 + 0.25 * m2[r];
    qr[r] = even + 0.5 * m1[r];
    ql[r] = even - 0.5 * m1[r];
    beta[r] = m1[r] * m1[r] + (13.0 / 3.0) * (m2[r] * m2[r]);
  }
  const double s0 = eps + beta[0], s1 = eps + beta[1], s2 = eps + beta[2];
  const double t0 = s0 * s0, t1 = s1 * s1, t2 = s2 * s2;
  const double p[3] = {t1 * t2, t0 * t2, t0 * t1};
  double wr[3], wl[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    wr[r] = cf[(NU_DR + r) * st] * p[r];
    wl[r] = cf[(NU_DL + r) * st] * p[r];
  }
  const double sr = wr[0] + wr[1] + wr[2], sl = wl[0] + wl[1] + wl[2];
  const double inv = fast_rcp(sr * sl);
  const double isr = sl * inv, isl = sr * inv;
  double cR = 0.0, cL = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    wr[r] *= isr;
    wl[r] *= isl;
    cR += wr[r] * qr[r];
    cL += wl[r] * ql[r];
  }
  const double sv[3] = {s0, s1, s2};
  double Db[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double qrb = gR * wr[r], qlb = gL * wl[r];
    const double bb = -2.0 * fast_rcp(sv[r]) * (qrb * (qr[r] - cR) + qlb * (ql[r] - cL));
    const double mu0b = qrb + qlb;
    const double m1b = 0.5 * (qrb - qlb) + 2.0 * m1[r] * bb;
    const double m2b = 0.25 * (qrb + qlb) + (26.0 / 3.0) * m2[r] * bb;
    Db[r] += cf[(NU_MU0 + 2 * r) * st] * mu0b + cf[(NU_M1 + 2 * r) * st] * m1b + cf[(NU_M2 + 2 * r) * st] * m2b;
    Db[r + 1] += cf[(NU_MU0 + 2 * r + 1) * st] * mu0b + cf[(NU_M1 + 2 * r + 1) * st] * m1b +
                 cf[(NU_M2 + 2 * r + 1) * st] * m2b;
  }
  g[2] += gR + gL;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    g[k + 1] += Db[k];
    g[k] -= Db[k];
  }
}

// ---------------------------------------------------------------------------
// HLLC adjoint (same readings as hllc()): given Fbar (every row) and ufbar,
// accumulate WLbar and WRbar.  Double precision.
// ---------------------------------------------------------------------------
template <int NF, int D>
struct SideState {
  double rho, Gam, Pi, p, un, usq, E, c2, c;
};

template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void side_state(const Params& pm, const double* W, SideState<NF, D>& s) {
  using R = Rows<NF, D>;
  s.rho = W[0];
  if constexpr (NF == 2) s.rho = W[0] + W[1];
  if constexpr (NF == 2)
    mixture<NF, double>(pm, W[R::ALPHA], W[R::ALPHA + 1], s.Gam, s.Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, s.Gam, s.Pi);
  s.p = W[R::E];
  s.un = W[R::MOM + DIR];
  s.usq = 0.0;
#pragma unroll
  for (int e = 0; e < D; ++e) s.usq += W[R::MOM + e] * W[R::MOM + e];
  s.E = s.Gam * s.p + s.Pi + 0.5 * s.rho * s.usq;
  s.c2 = sound_speed_sq(s.rho, s.p, s.Gam, s.Pi);
  s.c = sqrt(s.c2);
}

// Cotangents of the side scalars, pushed to the primitive cotangents of that side.
template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void side_scalars_vjp(const Params& pm, const double* W, const SideState<NF, D>& s,
                                                          double rhob, double Gamb, double Pib, double pb, double unb,
                                                          double Eb, double cb, double* Wb) {
  using R = Rows<NF, D>;
  // E = Gamma p + Pi + rho usq / 2
  Gamb += Eb * s.p;
  pb += Eb * s.Gam;
  Pib += Eb;
  rhob += Eb * 0.5 * s.usq;
  // c = sqrt(c2), c2 = ((Gamma + 1) p + Pi)/(Gamma rho)
  if (cb != 0.0) {
    const double c2b = 0.5 * cb * fast_rcp(s.c);
    const double rden = fast_rcp(s.Gam * s.rho);
    const double Nb = c2b * rden;
    const double Db = -c2b * s.c2 * rden;
    Gamb += Nb * s.p + Db * s.rho;
    pb += Nb * (s.Gam + 1.0);
    Pib += Nb;
    rhob += Db * s.Gam;
  }
#pragma unroll
  for (int e = 0; e < D; ++e) Wb[R::MOM + e] += Eb * s.rho * W[R::MOM + e];
  Wb[R::MOM + DIR] += unb;
  Wb[R::E] += pb;
#pragma unroll
  for (int i = 0; i < NF; ++i) Wb[i] += rhob;
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) Wb[R::ALPHA + j] += Gamb * pm.G[j] + Pib * pm.P[j];
  }
}

template <int NF, int D, int DIR, bool APC = false>
__host__ __device__ __forceinline__ void hllc_vjp(const Params& pm, const double* WL, const double* WR,
                                                  const double* Fb, double ufb, double* WLb, double* WRb,
                                                  double* uf_out = nullptr) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  SideState<NF, D> L, Rs;
  side_state<NF, D, DIR>(pm, WL, L);
  side_state<NF, D, DIR>(pm, WR, Rs);
  const double sla = L.un - L.c, slb = Rs.un - Rs.c, sra = L.un + L.c, srb = Rs.un + Rs.c;
  const bool sl_left = sla <= slb;
  const bool sr_left = sra >= srb;
  const double SL = sl_left ? sla : slb;
  const double SR = sr_left ? sra : srb;
  const double aL = SL - L.un, aR = SR - Rs.un;
  const double num = (Rs.p - L.p) + L.rho * L.un * aL - Rs.rho * Rs.un * aR;
  // S* = num / den with den = rho_L a_L - rho_R a_R < 0, formed as in the
  // forward solver: num * -(1 / -den)
  const double rnd = fast_rcp(Rs.rho * aR - L.rho * aL);
  const double Sstar = num * -rnd;
  const bool useL = (SL >= 0.0) || (Sstar >= 0.0);
  const bool star = useL ? !(SL >= 0.0) : (SR > 0.0);
  // the side K the face takes, selected element by element (no pointer select)
  double W[NEQ], Wk[NEQ];
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    W[v] = useL ? WL[v] : WR[v];
    Wk[v] = 0.0;
  }
  const double Krho = useL ? L.rho : Rs.rho;
  const double Kp = useL ? L.p : Rs.p;
  const double Kun = useL ? L.un : Rs.un;
  const double KE = useL ? L.E : Rs.E;
  const double SK = useL ? SL : SR;
  const double uf = star ? Sstar : Kun;
  if (uf_out) *uf_out = uf;

  // side-K scalar cotangents
  double rhob = 0.0, Gamb = 0.0, Pib = 0.0, pb = 0.0, unb = 0.0, Eb = 0.0;
  double Sstarb = 0.0, SKb = 0.0;

  // volume-fraction flux alpha_j u_f
  double ufb_tot = ufb;
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      ufb_tot += Fb[R::ALPHA + j] * W[R::ALPHA + j];
      Wk[R::ALPHA + j] += Fb[R::ALPHA + j] * uf;
    }
  }
  if (star)
    Sstarb += ufb_tot;
  else
    unb += ufb_tot;

  // physical flux of side K: F_i = arho_i un, F_m = rho u_e un + p (e == DIR), F_E = (E + p) un
  {
    double unb_f = 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      Wk[i] += Fb[i] * Kun;
      unb_f += Fb[i] * W[i];
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const double m = Krho * W[R::MOM + e];
      const double mb = Fb[R::MOM + e] * Kun;
      unb_f += Fb[R::MOM + e] * m;
      rhob += mb * W[R::MOM + e];
      Wk[R::MOM + e] += mb * Krho;
    }
    pb += Fb[R::MOM + DIR];
    unb_f += Fb[R::E] * (KE + Kp);
    Eb += Fb[R::E] * Kun;
    pb += Fb[R::E] * Kun;
    unb += unb_f;
  }

  if (star) {
    // F = F_K + S_K (U* - U), U* = chi (U with u_DIR -> S*, E -> G)
    const double A = SK - Kun;
    const double B = SK - Sstar;
    const double rA = fast_rcp(A), rB = fast_rcp(B);
    const double chi = A * rB;
    const double h = Krho * Sstar + Kp * rA;
    const double G = KE + (Sstar - Kun) * h;
    double chib = 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const double Ui = W[i];
      SKb += Fb[i] * (chi * Ui - Ui);
      const double Usb = SK * Fb[i];
      Wk[i] += -SK * Fb[i] + Usb * chi;
      chib += Usb * Ui;
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const double ue = W[R::MOM + e];
      const double m = Krho * ue;
      const double Us = (e == DIR) ? chi * Krho * Sstar : chi * Krho * ue;
      SKb += Fb[R::MOM + e] * (Us - m);
      const double Usb = SK * Fb[R::MOM + e];
      const double mb = -SK * Fb[R::MOM + e];
      rhob += mb * ue;
      Wk[R::MOM + e] += mb * Krho;
      if (e == DIR) {
        chib += Usb * Krho * Sstar;
        rhob += Usb * chi * Sstar;
        Sstarb += Usb * chi * Krho;
      } else {
        chib += Usb * Krho * ue;
        rhob += Usb * chi * ue;
        Wk[R::MOM + e] += Usb * chi * Krho;
      }
    }
    {
      SKb += Fb[R::E] * (chi * G - KE);
      const double Usb = SK * Fb[R::E];
      Eb += -SK * Fb[R::E];
      chib += Usb * G;
      const double Gb = Usb * chi;
      Eb += Gb;
      Sstarb += Gb * h;
      unb -= Gb * h;
      const double hb = Gb * (Sstar - Kun);
      rhob += hb * Sstar;
      Sstarb += hb * Krho;
      pb += hb * rA;
      // h holds p / A; chi = A / B
      const double Ab = -hb * Kp * (rA * rA) + chib * rB;
      const double Bb = -chib * chi * rB;
      SKb += Ab + Bb;
      unb -= Ab;
      Sstarb -= Bb;
    }
  }

  // APC term of Chen et al. in the star region: A = (z - 1) p_d on the normal
  // momentum and A S* on the energy, p_d = P / den2 with P = rho_L rho_R a_L
  // a_R (u_R - u_L), den2 = rho_R a_R - rho_L a_L (= 1/rnd); z = |u|/c of the
  // side the max took (ties: left), no derivative when clipped at 1
  double rhoLb = 0.0, unLb = 0.0, pLb = 0.0, cLb = 0.0;
  double rhoRb = 0.0, unRb = 0.0, pRb = 0.0, cRb = 0.0;
  double SLb = 0.0, SRb = 0.0;
  if constexpr (APC) {
    if (star) {
      const double mL = fabs(L.un) * fast_rcp(L.c), mR = fabs(Rs.un) * fast_rcp(Rs.c);
      const bool zleft = mL >= mR;
      const double zm = zleft ? mL : mR;
      const bool clipped = zm > 1.0;
      const double z = clipped ? 1.0 : zm;
      const double du = Rs.un - L.un;
      const double rr = L.rho * Rs.rho;
      const double pd = rr * aL * aR * du * rnd;
      const double Ab = Fb[R::MOM + DIR] + Fb[R::E] * Sstar;
      Sstarb += Fb[R::E] * ((z - 1.0) * pd);
      const double zb = Ab * pd;
      const double pdb = Ab * (z - 1.0);
      const double Pb = pdb * rnd;
      const double den2b = -pdb * pd * rnd;
      rhoLb += Pb * Rs.rho * aL * aR * du - den2b * aL;
      rhoRb += Pb * L.rho * aL * aR * du + den2b * aR;
      const double aLb = Pb * rr * aR * du - den2b * L.rho;
      const double aRb = Pb * rr * aL * du + den2b * Rs.rho;
      const double dub = Pb * rr * aL * aR;
      unRb += dub - aRb;
      unLb -= dub + aLb;
      SLb += aLb;
      SRb += aRb;
      if (!clipped) {
        if (zleft) {
          const double rc = fast_rcp(L.c);
          unLb += zb * ((L.un > 0.0) ? rc : ((L.un < 0.0) ? -rc : 0.0));
          cLb -= zb * fabs(L.un) * rc * rc;
        } else {
          const double rc = fast_rcp(Rs.c);
          unRb += zb * ((Rs.un > 0.0) ? rc : ((Rs.un < 0.0) ? -rc : 0.0));
          cRb -= zb * fabs(Rs.un) * rc * rc;
        }
      }
    }
  }

  // wave speeds: S* = num/den, S_L / S_R from the Davis estimates
  if (star) {
    if (useL)
      SLb += SKb;
    else
      SRb += SKb;
    const double numb = -Sstarb * rnd;          // Sstarb / den
    const double denb = Sstarb * Sstar * rnd;   // -Sstarb S* / den
    pRb += numb;
    pLb -= numb;
    rhoLb += numb * L.un * aL + denb * aL;
    unLb += numb * L.rho * aL;
    const double aLb = numb * L.rho * L.un + denb * L.rho;
    rhoRb -= numb * Rs.un * aR + denb * aR;
    unRb -= numb * Rs.rho * aR;
    const double aRb = -numb * Rs.rho * Rs.un - denb * Rs.rho;
    SLb += aLb;
    unLb -= aLb;
    SRb += aRb;
    unRb -= aRb;
    if (sl_left) {
      unLb += SLb;
      cLb -= SLb;
    } else {
      unRb += SLb;
      cRb -= SLb;
    }
    if (sr_left) {
      unLb += SRb;
      cLb += SRb;
    } else {
      unRb += SRb;
      cRb += SRb;
    }
  }
  // merge the selected side's own cotangents
  rhoLb += useL ? rhob : 0.0;
  unLb += useL ? unb : 0.0;
  pLb += useL ? pb : 0.0;
  rhoRb += useL ? 0.0 : rhob;
  unRb += useL ? 0.0 : unb;
  pRb += useL ? 0.0 : pb;
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    WLb[v] += useL ? Wk[v] : 0.0;
    WRb[v] += useL ? 0.0 : Wk[v];
  }
  side_scalars_vjp<NF, D, DIR>(pm, WL, L, rhoLb, useL ? Gamb : 0.0, useL ? Pib : 0.0, pLb, unLb, useL ? Eb : 0.0,
                               cLb, WLb);
  side_scalars_vjp<NF, D, DIR>(pm, WR, Rs, rhoRb, useL ? 0.0 : Gamb, useL ? 0.0 : Pib, pRb, unRb,
                               useL ? 0.0 : Eb, cRb, WRb);
}

// ---------------------------------------------------------------------------
// HLL adjoint (same readings as hll()).  Forward, per face:
//   F_v = N_v r, N_v = a F_L,v + b F_R,v + c (U_R,v - U_L,v), u_f = (a u_L + b u_R) r,
// (a, b, c, r) = (1, 0, 0, 1) | (0, 1, 0, 1) | (S_R, -S_L, S_L S_R, 1/(S_R - S_L)).
// With G_v = Fbar_v r the sides receive Fbar_L = a G, Fbar_R = b G,
// Ubar_R = c G, Ubar_L = -c G; between the waves the coefficients add
//   abar = sum G F_L + ufbar r u_L, bbar = sum G F_R + ufbar r u_R,
//   cbar = sum G (U_R - U_L), rbar = sum Fbar N + ufbar (a u_L + b u_R),
//   S_R bar = abar + cbar S_L - rbar r^2, S_L bar = -bbar + cbar S_R + rbar r^2,
// which reach u and c of the side each min / max took (ties: first).
// Accumulates WLbar, WRbar; uf_out (optional) receives the forward u_f.
// ---------------------------------------------------------------------------
template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void hll_side_rows_vjp(const double* W, const SideState<NF, D>& s,
                                                          const double* Fb, const double* Ub, double& rhob,
                                                          double& pb, double& unb, double& Eb, double* Wb) {
  using R = Rows<NF, D>;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    Wb[i] += Fb[i] * s.un + Ub[i];
    unb += Fb[i] * W[i];
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    const double m = s.rho * W[R::MOM + e];
    const double mb = Fb[R::MOM + e] * s.un + Ub[R::MOM + e];
    unb += Fb[R::MOM + e] * m;
    if (e == DIR) pb += Fb[R::MOM + e];
    rhob += mb * W[R::MOM + e];
    Wb[R::MOM + e] += mb * s.rho;
  }
  Eb += Fb[R::E] * s.un + Ub[R::E];
  pb += Fb[R::E] * s.un;
  unb += Fb[R::E] * (s.E + s.p);
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      Wb[R::ALPHA + j] += Fb[R::ALPHA + j] * s.un + Ub[R::ALPHA + j];
      unb += Fb[R::ALPHA + j] * W[R::ALPHA + j];
    }
  }
}

template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void hll_vjp(const Params& pm, const double* WL, const double* WR,
                                                 const double* Fb, double ufb, double* WLb, double* WRb,
                                                 double* uf_out = nullptr) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  SideState<NF, D> L, Rs;
  side_state<NF, D, DIR>(pm, WL, L);
  side_state<NF, D, DIR>(pm, WR, Rs);
  const double sla = L.un - L.c, slb = Rs.un - Rs.c, sra = L.un + L.c, srb = Rs.un + Rs.c;
  const bool sl_left = sla <= slb;
  const bool sr_left = sra >= srb;
  const double SL = sl_left ? sla : slb;
  const double SR = sr_left ? sra : srb;
  const bool lo = SL >= 0.0, hi = !lo && SR <= 0.0, mid = !lo && !hi;
  double a = 1.0, b = 0.0, c = 0.0, r = 1.0;
  if (hi) {
    a = 0.0;
    b = 1.0;
  } else if (mid) {
    a = SR;
    b = -SL;
    c = SL * SR;
    r = fast_rcp(SR - SL);
  }
  if (uf_out) *uf_out = (a * L.un + b * Rs.un) * r;
  // per-row physical fluxes and conservative values of both sides
  double FL[NEQ], FR[NEQ], UL[NEQ], UR[NEQ];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    UL[i] = WL[i];
    UR[i] = WR[i];
    FL[i] = WL[i] * L.un;
    FR[i] = WR[i] * Rs.un;
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    UL[R::MOM + e] = L.rho * WL[R::MOM + e];
    UR[R::MOM + e] = Rs.rho * WR[R::MOM + e];
    FL[R::MOM + e] = UL[R::MOM + e] * L.un + ((e == DIR) ? L.p : 0.0);
    FR[R::MOM + e] = UR[R::MOM + e] * Rs.un + ((e == DIR) ? Rs.p : 0.0);
  }
  UL[R::E] = L.E;
  UR[R::E] = Rs.E;
  FL[R::E] = (L.E + L.p) * L.un;
  FR[R::E] = (Rs.E + Rs.p) * Rs.un;
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      UL[R::ALPHA + j] = WL[R::ALPHA + j];
      UR[R::ALPHA + j] = WR[R::ALPHA + j];
      FL[R::ALPHA + j] = WL[R::ALPHA + j] * L.un;
      FR[R::ALPHA + j] = WR[R::ALPHA + j] * Rs.un;
    }
  }
  double FLb[NEQ], FRb[NEQ], ULb[NEQ], URb[NEQ];
  double ab = ufb * r * L.un, bb = ufb * r * Rs.un, cb = 0.0, rb = ufb * (a * L.un + b * Rs.un);
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    const double G = Fb[v] * r;
    const double dU = UR[v] - UL[v];
    FLb[v] = a * G;
    FRb[v] = b * G;
    URb[v] = c * G;
    ULb[v] = -c * G;
    ab += G * FL[v];
    bb += G * FR[v];
    cb += G * dU;
    rb += Fb[v] * (a * FL[v] + b * FR[v] + c * dU);
  }
  double unLb = ufb * r * a, unRb = ufb * r * b;
  double cLb = 0.0, cRb = 0.0;
  if (mid) {
    const double r2 = r * r;
    const double SRb = ab + cb * SL - rb * r2;
    const double SLb = -bb + cb * SR + rb * r2;
    if (sl_left) {
      unLb += SLb;
      cLb -= SLb;
    } else {
      unRb += SLb;
      cRb -= SLb;
    }
    if (sr_left) {
      unLb += SRb;
      cLb += SRb;
    } else {
      unRb += SRb;
      cRb += SRb;
    }
  }
  double rhoLb = 0.0, pLb = 0.0, ELb = 0.0, rhoRb = 0.0, pRb = 0.0, ERb = 0.0;
  hll_side_rows_vjp<NF, D, DIR>(WL, L, FLb, ULb, rhoLb, pLb, unLb, ELb, WLb);
  hll_side_rows_vjp<NF, D, DIR>(WR, Rs, FRb, URb, rhoRb, pRb, unRb, ERb, WRb);
  side_scalars_vjp<NF, D, DIR>(pm, WL, L, rhoLb, 0.0, 0.0, pLb, unLb, ELb, cLb, WLb);
  side_scalars_vjp<NF, D, DIR>(pm, WR, Rs, rhoRb, 0.0, 0.0, pRb, unRb, ERb, cRb, WRb);
}

// Adjoint of the low-Mach correction (thornber() in device.h).  Given the
// cotangents WLb, WRb of the corrected states (which differ from the states
// as reconstructed only in the normal velocity, so their sound speeds are
// those of the originals) and the original normal velocities uL, uR, turn
// WLb, WRb into the cotangents of the states as reconstructed:
//   uL* = (1 + z)/2 uL + (1 - z)/2 uR,  uR* = (1 - z)/2 uL + (1 + z)/2 uR,
//   zbar = (uL - uR)/2 (uL*bar - uR*bar), none when z is clipped at 1, to the
//   Mach number the max took (ties: first), and M = |u|/c gives u sign(u)/c and
//   c -|u|/c^2, pushed through the side-scalar adjoint.
template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void thornber_vjp(const Params& pm, const double* WL, const double* WR,
                                                      double uL, double uR, double* WLb, double* WRb) {
  using R = Rows<NF, D>;
  SideState<NF, D> L, Rs;
  side_state<NF, D, DIR>(pm, WL, L);
  side_state<NF, D, DIR>(pm, WR, Rs);
  const double mL = fabs(uL) / L.c, mR = fabs(uR) / Rs.c;
  const bool left = mL >= mR;
  const double zm = left ? mL : mR;
  const bool clipped = zm > 1.0;
  const double z = clipped ? 1.0 : zm;
  const double gl = WLb[R::MOM + DIR], gr = WRb[R::MOM + DIR];
  WLb[R::MOM + DIR] = 0.5 * (1.0 + z) * gl + 0.5 * (1.0 - z) * gr;
  WRb[R::MOM + DIR] = 0.5 * (1.0 - z) * gl + 0.5 * (1.0 + z) * gr;
  if (clipped) return;
  const double zb = 0.5 * (uL - uR) * (gl - gr);
  if (left) {
    const double rc = 1.0 / L.c;
    WLb[R::MOM + DIR] += zb * ((uL > 0.0) ? rc : ((uL < 0.0) ? -rc : 0.0));
    side_scalars_vjp<NF, D, DIR>(pm, WL, L, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -zb * fabs(uL) * rc * rc, WLb);
  } else {
    const double rc = 1.0 / Rs.c;
    WRb[R::MOM + DIR] += zb * ((uR > 0.0) ? rc : ((uR < 0.0) ? -rc : 0.0));
    side_scalars_vjp<NF, D, DIR>(pm, WR, Rs, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -zb * fabs(uR) * rc * rc, WRb);
  }
}

// The face-solver adjoint of a kernel instantiation (option bits RS as for
// riemann()): HLL, or HLLC with or without the APC term.
template <int RS, int NF, int D, int DIR>
__host__ __device__ __forceinline__ void riemann_vjp(const Params& pm, const double* WL, const double* WR,
                                                     const double* Fb, double ufb, double* WLb, double* WRb,
                                                     double* uf_out = nullptr) {
  if constexpr ((RS & RS_HLL) != 0)
    hll_vjp<NF, D, DIR>(pm, WL, WR, Fb, ufb, WLb, WRb, uf_out);
  else
    hllc_vjp<NF, D, DIR, (RS & RS_APC) != 0>(pm, WL, WR, Fb, ufb, WLb, WRb, uf_out);
}

// Gradient of Kapila's K (kapila_K) with respect to the cell's p, alpha_1 and
// alpha_2.  With z_i = gamma_i (p + pi_inf,i), N = z_2 - z_1, Q = z_1 alpha_2 +
// z_2 alpha_1 and K = N alpha_1 alpha_2 / Q:
//   dK/dp = ((gamma_2 - gamma_1) alpha_1 alpha_2 - K (gamma_1 alpha_2 + gamma_2 alpha_1)) / Q,
//   dK/dalpha_1 = (N alpha_2 - K z_2) / Q,  dK/dalpha_2 = (N alpha_1 - K z_1) / Q.
__host__ __device__ __forceinline__ void kapila_K_grad(const Params& pm, double p, double a1, double a2, double& dp,
                                                       double& da1, double& da2) {
  const double z1 = pm.gam[0] * (p + pm.pinf[0]);
  const double z2 = pm.gam[1] * (p + pm.pinf[1]);
  const double N = z2 - z1;
  const double rQ = fast_rcp(z1 * a2 + z2 * a1);
  const double K = N * (a1 * a2) * rQ;
  dp = ((pm.gam[1] - pm.gam[0]) * (a1 * a2) - K * (pm.gam[0] * a2 + pm.gam[1] * a1)) * rQ;
  da1 = (N * a2 - K * z2) * rQ;
  da2 = (N * a1 - K * z1) * rQ;
}

}  // namespace mfc
