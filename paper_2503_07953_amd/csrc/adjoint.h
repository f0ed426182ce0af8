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
  const double rinv = 1.0 / rho;
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
  const double p = (U[R::E] - 0.5 * rho * usq - Pi) / Gam;
  const double pb = wbar[R::E];
  const double gi = 1.0 / Gam;
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

// Adjoint of the left-biased WENO5-JS value at i+1/2 from f = (a, b, c, d, e):
// y = sum_k a_k q_k / sum_k a_k, a_k = d_k/(eps + beta_k)^2.  Accumulates g[0..4].
__host__ __device__ __forceinline__ void weno_left_vjp(double a, double b, double c, double d, double e,
                                                       double eps, double gy, double* g) {
  const double u0 = (a + c) - 2.0 * b, v0 = (a + 3.0 * c) - 4.0 * b;
  const double u1 = (b + d) - 2.0 * c, v1 = b - d;
  const double u2 = (c + e) - 2.0 * d, v2 = (3.0 * c + e) - 4.0 * d;
  const double s0 = eps + ((13.0 / 12.0) * u0 * u0 + 0.25 * v0 * v0);
  const double s1 = eps + ((13.0 / 12.0) * u1 * u1 + 0.25 * v1 * v1);
  const double s2 = eps + ((13.0 / 12.0) * u2 * u2 + 0.25 * v2 * v2);
  const double a0 = 0.1 / (s0 * s0), a1 = 0.6 / (s1 * s1), a2 = 0.3 / (s2 * s2);
  const double S = a0 + a1 + a2;
  const double Si = 1.0 / S;
  const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  const double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  const double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  const double y = (a0 * q0 + a1 * q1 + a2 * q2) * Si;
  // candidate values
  const double q0b = gy * a0 * Si, q1b = gy * a1 * Si, q2b = gy * a2 * Si;
  // weights -> smoothness indicators: d a_k / d beta_k = -2 a_k / s_k
  const double b0b = gy * (q0 - y) * Si * (-2.0 * a0 / s0);
  const double b1b = gy * (q1 - y) * Si * (-2.0 * a1 / s1);
  const double b2b = gy * (q2 - y) * Si * (-2.0 * a2 / s2);
  const double k = 13.0 / 6.0;
  g[0] += b0b * (k * u0 + 0.5 * v0) + q0b * (2.0 / 6.0);
  g[1] += b0b * (-2.0 * k * u0 - 2.0 * v0) + b1b * (k * u1 + 0.5 * v1) + q0b * (-7.0 / 6.0) - q1b * (1.0 / 6.0);
  g[2] += b0b * (k * u0 + 1.5 * v0) + b1b * (-2.0 * k * u1) + b2b * (k * u2 + 1.5 * v2) + q0b * (11.0 / 6.0) +
          q1b * (5.0 / 6.0) + q2b * (2.0 / 6.0);
  g[3] += b1b * (k * u1 - 0.5 * v1) + b2b * (-2.0 * k * u2 - 2.0 * v2) + q1b * (2.0 / 6.0) + q2b * (5.0 / 6.0);
  g[4] += b2b * (k * u2 + 0.5 * v2) - q2b * (1.0 / 6.0);
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
    const double c2b = cb / (2.0 * s.c);
    const double den = s.Gam * s.rho;
    const double Nb = c2b / den;
    const double Db = -c2b * s.c2 / den;
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

template <int NF, int D, int DIR>
__host__ __device__ __forceinline__ void hllc_vjp(const Params& pm, const double* WL, const double* WR,
                                                  const double* Fb, double ufb, double* WLb, double* WRb) {
  using R = Rows<NF, D>;
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
  const double den = L.rho * aL - Rs.rho * aR;
  const double Sstar = num / den;
  const bool useL = (SL >= 0.0) || (Sstar >= 0.0);
  const bool star = useL ? !(SL >= 0.0) : (SR > 0.0);
  const double* W = useL ? WL : WR;
  double* Wb = useL ? WLb : WRb;
  const SideState<NF, D>& K = useL ? L : Rs;
  const double SK = useL ? SL : SR;
  const double uf = star ? Sstar : K.un;

  // side-K scalar cotangents
  double rhob = 0.0, Gamb = 0.0, Pib = 0.0, pb = 0.0, unb = 0.0, Eb = 0.0;
  double Sstarb = 0.0, SKb = 0.0;

  // volume-fraction flux alpha_j u_f
  double ufb_tot = ufb;
  if constexpr (NF == 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      ufb_tot += Fb[R::ALPHA + j] * W[R::ALPHA + j];
      Wb[R::ALPHA + j] += Fb[R::ALPHA + j] * uf;
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
      Wb[i] += Fb[i] * K.un;
      unb_f += Fb[i] * W[i];
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const double m = K.rho * W[R::MOM + e];
      const double mb = Fb[R::MOM + e] * K.un;
      unb_f += Fb[R::MOM + e] * m;
      rhob += mb * W[R::MOM + e];
      Wb[R::MOM + e] += mb * K.rho;
    }
    pb += Fb[R::MOM + DIR];
    unb_f += Fb[R::E] * (K.E + K.p);
    Eb += Fb[R::E] * K.un;
    pb += Fb[R::E] * K.un;
    unb += unb_f;
  }

  if (star) {
    // F = F_K + S_K (U* - U)
    const double A = SK - K.un;
    const double B = SK - Sstar;
    const double chi = A / B;
    const double h = K.rho * Sstar + K.p / A;
    const double G = K.E + (Sstar - K.un) * h;
    double chib = 0.0;
    // S_K (U* - U): cotangent of S_K, of U* and of U
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const double Ui = W[i];
      const double Us = chi * Ui;
      SKb += Fb[i] * (Us - Ui);
      const double Usb = SK * Fb[i];
      Wb[i] += -SK * Fb[i] + Usb * chi;
      chib += Usb * Ui;
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const double ue = W[R::MOM + e];
      const double m = K.rho * ue;
      const double Us = (e == DIR) ? chi * K.rho * Sstar : chi * K.rho * ue;
      SKb += Fb[R::MOM + e] * (Us - m);
      const double Usb = SK * Fb[R::MOM + e];
      const double mb = -SK * Fb[R::MOM + e];
      rhob += mb * ue;
      Wb[R::MOM + e] += mb * K.rho;
      if (e == DIR) {
        chib += Usb * K.rho * Sstar;
        rhob += Usb * chi * Sstar;
        Sstarb += Usb * chi * K.rho;
      } else {
        chib += Usb * K.rho * ue;
        rhob += Usb * chi * ue;
        Wb[R::MOM + e] += Usb * chi * K.rho;
      }
    }
    {
      const double Us = chi * G;
      SKb += Fb[R::E] * (Us - K.E);
      const double Usb = SK * Fb[R::E];
      Eb += -SK * Fb[R::E];
      chib += Usb * G;
      const double Gb = Usb * chi;
      Eb += Gb;
      Sstarb += Gb * h;
      unb -= Gb * h;
      const double hb = Gb * (Sstar - K.un);
      rhob += hb * Sstar;
      Sstarb += hb * K.rho;
      pb += hb / A;
      double Ab = -hb * K.p / (A * A);
      // chi = A / B
      Ab += chib / B;
      const double Bb = -chib * A / (B * B);
      SKb += Ab + Bb;
      unb -= Ab;
      Sstarb -= Bb;
    }
  }

  // wave speeds: S* = num/den, S_L / S_R from the Davis estimates
  double rhoLb = 0.0, unLb = 0.0, pLb = 0.0, cLb = 0.0;
  double rhoRb = 0.0, unRb = 0.0, pRb = 0.0, cRb = 0.0;
  double SLb = 0.0, SRb = 0.0;
  if (star) {
    if (useL)
      SLb += SKb;
    else
      SRb += SKb;
    const double numb = Sstarb / den;
    const double denb = -Sstarb * Sstar / den;
    pRb += numb;
    pLb -= numb;
    rhoLb += numb * L.un * aL + denb * aL;
    unLb += numb * L.rho * aL;
    double aLb = numb * L.rho * L.un + denb * L.rho;
    rhoRb -= numb * Rs.un * aR + denb * aR;
    unRb -= numb * Rs.rho * aR;
    double aRb = -numb * Rs.rho * Rs.un - denb * Rs.rho;
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
  if (useL) {
    rhoLb += rhob;
    unLb += unb;
    pLb += pb;
  } else {
    rhoRb += rhob;
    unRb += unb;
    pRb += pb;
  }
  side_scalars_vjp<NF, D, DIR>(pm, WL, L, rhoLb, useL ? Gamb : 0.0, useL ? Pib : 0.0, pLb, unLb, useL ? Eb : 0.0,
                               cLb, WLb);
  side_scalars_vjp<NF, D, DIR>(pm, WR, Rs, rhoRb, useL ? 0.0 : Gamb, useL ? 0.0 : Pib, pRb, unRb,
                               useL ? 0.0 : Eb, cRb, WRb);
}

}  // namespace mfc
