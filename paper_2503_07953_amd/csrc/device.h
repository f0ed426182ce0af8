// device.h -- per-cell and per-face device arithmetic of the five-equation RHS
// for gfx950: stiffened-gas closure, ghost-layer index map, WENO5-JS and HLLC.
//
// Every function here is templated on the grid (fluid count NF, dimension D)
// so that row indices and loop trip counts are compile-time constants: the
// problem-specialized code generation the paper gets from its "case
// optimization" (Sec. 4.3.3) comes from C++ templates instead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfc {

enum { BC_PERIODIC = 0, BC_EXTRAP = 1, BC_SLIPWALL = 2 };

// Problem constants passed to every kernel by value.
struct Params {
  int n[3];            // interior cells per axis (unused axes: 1)
  int bc_lo[3];        // BC kind per axis, low side
  int bc_hi[3];        // BC kind per axis, high side
  int pad_;
  double inv_dx[3];    // 1/dx per axis
  double G[2];         // 1/(gamma_i - 1)
  double P[2];         // gamma_i pi_inf,i/(gamma_i - 1)
  double eps;          // WENO regularization
  long long ncell;     // nx*ny*nz: stride between rows
};

// Row layout for NF fluids in D dimensions.
template <int NF, int D>
struct Rows {
  static constexpr int NEQ = NF + D + 1 + (NF == 2 ? 2 : 0);
  static constexpr int MOM = NF;        // first momentum / velocity row
  static constexpr int E = NF + D;      // energy / pressure row
  static constexpr int ALPHA = NF + D + 1;  // first volume-fraction row (NF == 2)
  static constexpr int NCONS = NF + D + 1;  // rows with a conservative flux
};

// Index of the interior cell that ghost (or interior) index g along an axis of
// n cells maps to (Sec. 3.3 buffer layers): periodic wrap, zeroth-degree
// extrapolation, or mirror image for a slip wall (flip = normal momentum
// changes sign).  Valid for -3 <= g <= n + 2 with n >= 3.
__host__ __device__ __forceinline__ int ghost_index(int g, int n, int lo, int hi, bool& flip) {
  flip = false;
  if (g < 0) {
    if (lo == BC_PERIODIC) return g + n;
    if (lo == BC_EXTRAP) return 0;
    flip = true;
    return -1 - g;
  }
  if (g >= n) {
    if (hi == BC_PERIODIC) return g - n;
    if (hi == BC_EXTRAP) return n - 1;
    flip = true;
    return 2 * n - 1 - g;
  }
  return g;
}

// Mixture Gamma = sum alpha_i G_i and Pi = sum alpha_i P_i (Sec. 2.1.1 mixture
// rules with the stiffened-gas law of Sec. 2.2).  One fluid: alpha = 1.
template <int NF, typename T>
__host__ __device__ __forceinline__ void mixture(const Params& pm, T a0, T a1, T& Gam, T& Pi) {
  if constexpr (NF == 1) {
    Gam = T(pm.G[0]);
    Pi = T(pm.P[0]);
  } else {
    Gam = a0 * T(pm.G[0]) + a1 * T(pm.G[1]);
    Pi = a0 * T(pm.P[0]) + a1 * T(pm.P[1]);
  }
}

// Conservative -> primitive for one cell, in double (the pressure inversion
// from total energy stays in double in both precision forms):
// u = (rho u)/rho, p = (rho E - rho |u|^2/2 - Pi)/Gamma.
template <int NF, int D>
__host__ __device__ __forceinline__ void cons_to_prim(const Params& pm, const double* U, double* W) {
  using R = Rows<NF, D>;
  double rho = U[0];
  if constexpr (NF == 2) rho = U[0] + U[1];
  const double rinv = 1.0 / rho;
  double usq = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double u = U[R::MOM + d] * rinv;
    W[R::MOM + d] = u;
    usq += u * u;
  }
  double Gam, Pi;
  if constexpr (NF == 2)
    mixture<NF, double>(pm, U[R::ALPHA], U[R::ALPHA + 1], Gam, Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, Gam, Pi);
  W[R::E] = (U[R::E] - 0.5 * rho * usq - Pi) / Gam;
#pragma unroll
  for (int i = 0; i < NF; ++i) W[i] = U[i];
  if constexpr (NF == 2) {
    W[R::ALPHA] = U[R::ALPHA];
    W[R::ALPHA + 1] = U[R::ALPHA + 1];
  }
}

// Squared mixture sound speed, the mixture read as one stiffened gas with
// gamma_m = 1 + 1/Gamma, pi_m = Pi/(Gamma + 1): c^2 = ((Gamma+1) p + Pi)/(Gamma rho).
__host__ __device__ __forceinline__ double sound_speed_sq(double rho, double p, double Gam, double Pi) {
  return ((Gam + 1.0) * p + Pi) / (Gam * rho);
}

// ---------------------------------------------------------------------------
// WENO5-JS (Sec. 3.2.1, Jiang-Shu weights) at one reconstruction centre:
// from cell values a..e = f_{i-2..i+2}, fl is the left-biased value at
// i+1/2 and fr the right-biased value at i-1/2.  The three smoothness
// indicators are shared by both values (the right value is the mirror image
// of the left one, whose indicators are the same three numbers).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double sq(double x) { return x * x; }
__host__ __device__ __forceinline__ float sq(float x) { return x * x; }

// FP64: the normalized weights a_k/sum(a) with a_k = d_k/t_k, t_k =
// (eps + beta_k)^2 are rewritten over the common denominator t0 t1 t2, so
// a_k is proportional to d_k times the product of the other two t's; this
// needs one division per biased value instead of four.  The products stay far
// inside the double range (t <= ~1e40 for pressures of ~1e9 Pa).
__host__ __device__ __forceinline__ void weno5_js(double a, double b, double c, double d, double e,
                                         double eps, double& fl, double& fr) {
  const double b0 = (13.0 / 12.0) * sq((a + c) - 2.0 * b) + 0.25 * sq((a + 3.0 * c) - 4.0 * b);
  const double b1 = (13.0 / 12.0) * sq((b + d) - 2.0 * c) + 0.25 * sq(b - d);
  const double b2 = (13.0 / 12.0) * sq((c + e) - 2.0 * d) + 0.25 * sq((3.0 * c + e) - 4.0 * d);
  const double t0 = sq(eps + b0), t1 = sq(eps + b1), t2 = sq(eps + b2);
  const double p0 = t1 * t2, p1 = t0 * t2, p2 = t0 * t1;
  // six times the candidate values
  const double l0 = 2.0 * a - 7.0 * b + 11.0 * c;
  const double l1 = -b + 5.0 * c + 2.0 * d;
  const double l2 = 2.0 * c + 5.0 * d - e;
  const double r0 = 2.0 * e - 7.0 * d + 11.0 * c;
  const double r1 = -d + 5.0 * c + 2.0 * b;
  const double r2 = 2.0 * c + 5.0 * b - a;
  const double wl0 = 0.1 * p0, wl1 = 0.6 * p1, wl2 = 0.3 * p2;
  const double wr0 = 0.1 * p2, wr1 = 0.6 * p1, wr2 = 0.3 * p0;
  fl = (wl0 * l0 + wl1 * l1 + wl2 * l2) / (6.0 * (wl0 + wl1 + wl2));
  fr = (wr0 * r0 + wr1 * r1 + wr2 * r2) / (6.0 * (wr0 + wr1 + wr2));
}

// FP32: products of t's would overflow float for pressure-sized data, so the
// weights use hardware reciprocals of t_k (v_rcp_f32, ~1 ulp).
__device__ __forceinline__ void weno5_js(float a, float b, float c, float d, float e, float eps,
                                         float& fl, float& fr) {
  const float b0 = (13.0f / 12.0f) * sq((a + c) - 2.0f * b) + 0.25f * sq((a + 3.0f * c) - 4.0f * b);
  const float b1 = (13.0f / 12.0f) * sq((b + d) - 2.0f * c) + 0.25f * sq(b - d);
  const float b2 = (13.0f / 12.0f) * sq((c + e) - 2.0f * d) + 0.25f * sq((3.0f * c + e) - 4.0f * d);
  const float s0 = __builtin_amdgcn_rcpf(sq(eps + b0));
  const float s1 = __builtin_amdgcn_rcpf(sq(eps + b1));
  const float s2 = __builtin_amdgcn_rcpf(sq(eps + b2));
  const float l0 = 2.0f * a - 7.0f * b + 11.0f * c;
  const float l1 = -b + 5.0f * c + 2.0f * d;
  const float l2 = 2.0f * c + 5.0f * d - e;
  const float r0 = 2.0f * e - 7.0f * d + 11.0f * c;
  const float r1 = -d + 5.0f * c + 2.0f * b;
  const float r2 = 2.0f * c + 5.0f * b - a;
  const float wl0 = 0.1f * s0, wl1 = 0.6f * s1, wl2 = 0.3f * s2;
  const float wr0 = 0.1f * s2, wr1 = 0.6f * s1, wr2 = 0.3f * s0;
  fl = (wl0 * l0 + wl1 * l1 + wl2 * l2) * __builtin_amdgcn_rcpf(6.0f * (wl0 + wl1 + wl2));
  fr = (wr0 * r0 + wr1 * r1 + wr2 * r2) * __builtin_amdgcn_rcpf(6.0f * (wr0 + wr1 + wr2));
}

// ---------------------------------------------------------------------------
// HLLC face solver (Sec. 3.2.2; star states of Toro's book), returning the flux
// of every row and the face velocity u_f.  T is the flux arithmetic type;
// sound speeds and the wave speeds S_L, S_R, S* are always double.
//   S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R) (the form
//   printed for the HLLD solver, Sec. 4.2.6), ties to the first argument;
//   regions: S_L >= 0 left; S* >= 0 left star; S_R > 0 right star; else right;
//   volume fractions are carried by the contact: flux alpha_K u_f.
// Returns true when a side has c^2 <= 0 or a flux is not finite.
// ---------------------------------------------------------------------------
template <int NF, int D, int DIR, typename T>
__host__ __device__ __forceinline__ bool hllc(const Params& pm, const T* WL, const T* WR, T* F, T& uf) {
  using R = Rows<NF, D>;
  // side quantities
  T rhoL = WL[0], rhoR = WR[0];
  if constexpr (NF == 2) {
    rhoL = WL[0] + WL[1];
    rhoR = WR[0] + WR[1];
  }
  T GamL, PiL, GamR, PiR;
  if constexpr (NF == 2) {
    mixture<NF, T>(pm, WL[R::ALPHA], WL[R::ALPHA + 1], GamL, PiL);
    mixture<NF, T>(pm, WR[R::ALPHA], WR[R::ALPHA + 1], GamR, PiR);
  } else {
    mixture<NF, T>(pm, T(1), T(0), GamL, PiL);
    mixture<NF, T>(pm, T(1), T(0), GamR, PiR);
  }
  const T pL = WL[R::E], pR = WR[R::E];
  const T unL = WL[R::MOM + DIR], unR = WR[R::MOM + DIR];
  const double c2L = sound_speed_sq(double(rhoL), double(pL), double(GamL), double(PiL));
  const double c2R = sound_speed_sq(double(rhoR), double(pR), double(GamR), double(PiR));
  const double cL = sqrt(c2L), cR = sqrt(c2R);
  const double dunL = double(unL), dunR = double(unR);
  const double sla = dunL - cL, slb = dunR - cR, sra = dunL + cL, srb = dunR + cR;
  const double SL = (sla <= slb) ? sla : slb;
  const double SR = (sra >= srb) ? sra : srb;
  const double drhoL = double(rhoL), drhoR = double(rhoR);
  const double Sstar = (double(pR) - double(pL) + drhoL * dunL * (SL - dunL) - drhoR * dunR * (SR - dunR)) /
                       (drhoL * (SL - dunL) - drhoR * (SR - dunR));

  // side the face takes and whether it lies in the star region
  const bool useL = (SL >= 0.0) || (Sstar >= 0.0);
  const bool star = useL ? !(SL >= 0.0) : (SR > 0.0);
  T W[R::NEQ];
#pragma unroll
  for (int v = 0; v < R::NEQ; ++v) W[v] = useL ? WL[v] : WR[v];
  const T rho = useL ? rhoL : rhoR;
  const T Gam = useL ? GamL : GamR;
  const T Pi = useL ? PiL : PiR;
  const T p = useL ? pL : pR;
  const T un = useL ? unL : unR;
  const double SK = useL ? SL : SR;

  T usq = T(0);
#pragma unroll
  for (int e = 0; e < D; ++e) usq += W[R::MOM + e] * W[R::MOM + e];
  const T E = Gam * p + Pi + T(0.5) * rho * usq;

  // physical flux of side K, then the star correction F + S_K (U* - U)
  // star-region factors; outside the star region they are replaced by harmless
  // values so that a degenerate S_K - u_K or S_K - S* cannot poison the flux
  const double dun = double(un);
  const double skmu = star ? (SK - dun) : 1.0;
  const double chi = star ? skmu / (SK - Sstar) : 1.0;
  const T s = star ? T(SK) : T(0);
  const T chiT = T(chi);
  const T SstarT = T(Sstar);
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const T Ui = W[i];
    F[i] = Ui * un + s * (chiT * Ui - Ui);
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    const T m = rho * W[R::MOM + e];
    const T us = (e == DIR) ? chiT * rho * SstarT : chiT * rho * W[R::MOM + e];
    F[R::MOM + e] = m * un + ((e == DIR) ? p : T(0)) + s * (us - m);
  }
  {
    const T Es = chiT * (E + (SstarT - un) * (rho * SstarT + T(double(p) / skmu)));
    F[R::E] = (E + p) * un + s * (Es - E);
  }
  uf = star ? SstarT : un;
  if constexpr (NF == 2) {
    F[R::ALPHA] = W[R::ALPHA] * uf;
    F[R::ALPHA + 1] = W[R::ALPHA + 1] * uf;
  }
  // explicit class checks: an "x - x == 0" test would not survive fused
  // multiply-add contraction (a*b - a*b becomes the rounding residual)
  bool finite = isfinite(uf);
#pragma unroll
  for (int v = 0; v < R::NEQ; ++v) finite = finite && isfinite(F[v]);
  return !(c2L > 0.0 && c2R > 0.0 && finite);
}

}  // namespace mfc
