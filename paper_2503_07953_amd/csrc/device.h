// device.h -- per-cell and per-face device arithmetic of the five-equation RHS
// for gfx950: stiffened-gas closure, ghost-layer index map, WENO5-JS and HLLC.
//
// Every function here is templated on the grid (fluid count NF, dimension D)
// so that row indices and loop trip counts are compile-time constants: the
// problem-specialized code generation the paper gets from its "case
// optimization" (Sec. 4.3.6) comes from C++ templates instead.
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
  int weno_variant;    // 0: WENO5-JS, 1: WENO5-Z, 2: TENO5, 3: WENO5-M
  int riemann;         // 0: HLLC, 1: HLL (Sec. 3.2.2)
  int low_mach;        // 0: none, 1: Thornber et al. velocity correction, 2: Chen et al. APC
  int model;           // 0: Allaire (K = 0), 1: Kapila (K div u on the alpha rows)
  double inv_dx[3];    // 1/dx per axis
  double G[2];         // 1/(gamma_i - 1)
  double P[2];         // gamma_i pi_inf,i/(gamma_i - 1)
  double gam[2];       // gamma_i
  double pinf[2];      // pi_inf,i
  double eps;          // WENO regularization
  long long ncell;     // nx*ny*nz: stride between rows
  // Non-uniform grid (set by mfc_set_grid): per axis, a table of kNuCoefs rows
  // of n + 6 entries (positions -3 .. n + 2), in double and in float; null on
  // a uniform grid.
  const double* nu[3];
  const float* nuf[3];
};

// Rows of the non-uniform reconstruction table of one axis (entry pos + 3 for
// the centre cell at position pos).  In the centre cell's unit coordinate
// xi = (x - x_c)/h_c, candidate r (cells c - 2 + r .. c + r) is the quadratic
// m0 + m1 xi + m2 xi^2 whose cell averages are the data; with D_k = f_{k+1} -
// f_k over the five cells f_0 .. f_4 (centre f_2), m0 - f_2, m1 and m2 are
// combinations a D_r + b D_{r+1} of the stencil's two differences:
//   NU_MU0 + 2 r (+1): a, b of m0 - f_2;  NU_M1 + 2 r (+1): of m1;
//   NU_M2 + 2 r (+1): of m2;
//   NU_DR + r: ideal weight of candidate r at the right face (xi = 1/2);
//   NU_DL + r: at the left face (xi = -1/2);
//   NU_INVW: 1/h of the cell at that position.
enum { NU_MU0 = 0, NU_M1 = 6, NU_M2 = 12, NU_DR = 18, NU_DL = 21, NU_INVW = 24, kNuCoefs = 25 };

// 1/h of cell i along axis d (uniform or tabulated).
__host__ __device__ __forceinline__ double inv_width(const Params& pm, int d, int i) {
  return pm.nu[d] ? pm.nu[d][(long long)NU_INVW * (pm.n[d] + 6) + i + 3] : pm.inv_dx[d];
}

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

// Reciprocal of a positive normal double: hardware estimate (v_rcp_f64)
// refined by two Newton steps (relative error a few ulp; no IEEE division
// sequence).  The host compilation, used only to exercise this arithmetic on
// the CPU, starts the same refinement from an exact quotient.
__host__ __device__ __forceinline__ double fast_rcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
#else
  double r = 1.0 / x;
#endif
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Conservative -> primitive for one cell, in double (the pressure inversion
// from total energy stays in double in both precision forms):
// u = (rho u)/rho, p = (rho E - rho |u|^2/2 - Pi)/Gamma.
template <int NF, int D>
__host__ __device__ __forceinline__ void cons_to_prim(const Params& pm, const double* U, double* W) {
  using R = Rows<NF, D>;
  double rho = U[0];
  if constexpr (NF == 2) rho = U[0] + U[1];
  const double rinv = fast_rcp(rho);
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
  W[R::E] = (U[R::E] - 0.5 * rho * usq - Pi) * fast_rcp(Gam);
#pragma unroll
  for (int i = 0; i < NF; ++i) W[i] = U[i];
  if constexpr (NF == 2) {
    W[R::ALPHA] = U[R::ALPHA];
    W[R::ALPHA + 1] = U[R::ALPHA + 1];
  }
}

// Primitive -> conservative for one cell, in double: rho u = rho * u,
// rho E = Gamma p + Pi + rho |u|^2/2.
template <int NF, int D>
__host__ __device__ __forceinline__ void prim_to_cons(const Params& pm, const double* W, double* U) {
  using R = Rows<NF, D>;
  double rho = W[0];
  if constexpr (NF == 2) rho = W[0] + W[1];
  double usq = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    U[R::MOM + d] = rho * W[R::MOM + d];
    usq += W[R::MOM + d] * W[R::MOM + d];
  }
  double Gam, Pi;
  if constexpr (NF == 2)
    mixture<NF, double>(pm, W[R::ALPHA], W[R::ALPHA + 1], Gam, Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, Gam, Pi);
  U[R::E] = Gam * W[R::E] + Pi + 0.5 * rho * usq;
#pragma unroll
  for (int i = 0; i < NF; ++i) U[i] = W[i];
  if constexpr (NF == 2) {
    U[R::ALPHA] = W[R::ALPHA];
    U[R::ALPHA + 1] = W[R::ALPHA + 1];
  }
}

// Squared mixture sound speed, the mixture read as one stiffened gas with
// gamma_m = 1 + 1/Gamma, pi_m = Pi/(Gamma + 1): c^2 = ((Gamma+1) p + Pi)/(Gamma rho).
__host__ __device__ __forceinline__ double sound_speed_sq(double rho, double p, double Gam, double Pi) {
  return ((Gam + 1.0) * p + Pi) * fast_rcp(Gam * rho);
}

// Kapila's K of one cell (Sec. 2.1.1): the alpha_1 row carries
// (alpha_1 + K) div u and the alpha_2 row (alpha_2 - K) div u, with
//   K = (rho_2 c_2^2 - rho_1 c_1^2) / (rho_1 c_1^2/alpha_1 + rho_2 c_2^2/alpha_2)
// and phasic sound speeds c_i^2 = gamma_i (p + pi_inf,i)/rho_i, so that
// rho_i c_i^2 = gamma_i (p + pi_inf,i) needs no phasic density.  The numerator
// is the difference of the two phases' stiffnesses: K vanishes for identical
// fluids.  Double arithmetic from the cell's pressure and volume fractions,
// over the common denominator: K = (z_2 - z_1) alpha_1 alpha_2 / (z_1 alpha_2 +
// z_2 alpha_1) with z_i = gamma_i (p + pi_inf,i).
__host__ __device__ __forceinline__ double kapila_K(const Params& pm, double p, double a1, double a2) {
  const double z1 = pm.gam[0] * (p + pm.pinf[0]);
  const double z2 = pm.gam[1] * (p + pm.pinf[1]);
  return (z2 - z1) * (a1 * a2) * fast_rcp(z1 * a2 + z2 * a1);
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

// FP64 WENO5-JS in difference form.  With D0..D3 the differences of the
// five cell values (D_k = f_{k+1} - f_k), each candidate is the centre value
// c plus a correction (e.g. q0 = c + (5 D1 - 2 D0)/6) and each smoothness
// indicator is 13/12 u^2 + 1/4 v^2 with u, v two differences of differences;
// here 4*beta = (13/3) u^2 + v^2 is formed and eps scaled by 4 to match, which
// leaves the normalized weights unchanged.  The weights a_k = d_k/(eps +
// beta_k)^2 are taken over the common denominator t0 t1 t2 (t_k = (eps +
// beta_k)^2), so a_k is proportional to d_k times the product of the other two
// t's; the two normalizations share one refined reciprocal.  The products stay
// far inside the double range (t <= ~1e40 for pressure jumps of ~1e9 Pa).
__host__ __device__ __forceinline__ void weno5_js(double a, double b, double c, double d, double e,
                                                  double eps, double& fl, double& fr) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double t0 = s0 * s0, t1 = s1 * s1, t2 = s2 * s2;
  const double p0 = t1 * t2, p1 = t0 * t2, p2 = t0 * t1;
  // six times the candidate corrections
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double r0 = 2.0 * D3 - 5.0 * D2, r1 = -(D2 + 2.0 * D1), r2 = D0 - 4.0 * D1;
  const double w1 = 0.6 * p1;
  const double wl0 = 0.1 * p0, wl2 = 0.3 * p2;
  const double wr0 = 0.1 * p2, wr2 = 0.3 * p0;
  const double nl = wl0 * l0 + w1 * l1 + wl2 * l2;
  const double nr = wr0 * r0 + w1 * r1 + wr2 * r2;
  const double dl = wl0 + w1 + wl2;
  const double dr = wr0 + w1 + wr2;
  const double inv = fast_rcp(6.0 * (dl * dr));
  fl = c + nl * (dr * inv);
  fr = c + nr * (dl * inv);
}

// FP32: the same difference form.  Squared indicators overflow float for
// pressure jumps of a few GPa (s ~ 1e19, s^2 > 3.4e38), so the weights are
// formed from the ratios s_min/s_k in (0, 1] (hardware reciprocals, ~1 ulp):
// a_k = (s_min/s_k)^2 is d_k/(eps + beta_k)^2 up to the common factor s_min^2,
// which the normalization removes, and the largest a_k is exactly 1.  Each
// biased value has its own normalization.
__device__ __forceinline__ void weno5_js(float a, float b, float c, float d, float e, float eps,
                                         float& fl, float& fr) {
  const float D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const float u0 = D1 - D0, v0 = 3.0f * D1 - D0;
  const float u1 = D2 - D1, v1 = D1 + D2;
  const float u2 = D3 - D2, v2 = D3 - 3.0f * D2;
  const float e4 = 4.0f * eps;
  const float s0 = e4 + ((13.0f / 3.0f) * u0 * u0 + v0 * v0);
  const float s1 = e4 + ((13.0f / 3.0f) * u1 * u1 + v1 * v1);
  const float s2 = e4 + ((13.0f / 3.0f) * u2 * u2 + v2 * v2);
  const float sm = fminf(s0, fminf(s1, s2));
  const float a0 = sq(sm * __builtin_amdgcn_rcpf(s0));
  const float a1 = sq(sm * __builtin_amdgcn_rcpf(s1));
  const float a2 = sq(sm * __builtin_amdgcn_rcpf(s2));
  const float l0 = 5.0f * D1 - 2.0f * D0, l1 = D1 + 2.0f * D2, l2 = 4.0f * D2 - D3;
  const float r0 = 2.0f * D3 - 5.0f * D2, r1 = -(D2 + 2.0f * D1), r2 = D0 - 4.0f * D1;
  const float w1 = 0.6f * a1;
  const float wl0 = 0.1f * a0, wl2 = 0.3f * a2;
  const float wr0 = 0.1f * a2, wr2 = 0.3f * a0;
  fl = c + (wl0 * l0 + w1 * l1 + wl2 * l2) * __builtin_amdgcn_rcpf(6.0f * (wl0 + w1 + wl2));
  fr = c + (wr0 * r0 + w1 * r1 + wr2 * r2) * __builtin_amdgcn_rcpf(6.0f * (wr0 + w1 + wr2));
}

// WENO5-Z (Sec. 4.2.2): the same candidates and smoothness indicators, the
// global indicator tau = |beta_0 - beta_2| and weights d_k (1 + tau/(beta_k +
// eps)) (exponent q = 1).  With s_k = 4 (eps + beta_k) as above, tau' = |s_0 -
// s_2| = 4 tau and the weights are d_k (s_k + tau')/s_k; over the common
// denominator s_0 s_1 s_2 they become d_k (s_k + tau') prod_{j != k} s_j, so
// both biased values again need one refined reciprocal.
__host__ __device__ __forceinline__ void weno5_z(double a, double b, double c, double d, double e, double eps,
                                                 double& fl, double& fr) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double tau = fabs(s0 - s2);
  const double z0 = (s0 + tau) * (s1 * s2), z1 = (s1 + tau) * (s0 * s2), z2 = (s2 + tau) * (s0 * s1);
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double r0 = 2.0 * D3 - 5.0 * D2, r1 = -(D2 + 2.0 * D1), r2 = D0 - 4.0 * D1;
  const double w1 = 0.6 * z1;
  const double wl0 = 0.1 * z0, wl2 = 0.3 * z2;
  const double wr0 = 0.1 * z2, wr2 = 0.3 * z0;
  const double nl = wl0 * l0 + w1 * l1 + wl2 * l2;
  const double nr = wr0 * r0 + w1 * r1 + wr2 * r2;
  const double dl = wl0 + w1 + wl2;
  const double dr = wr0 + w1 + wr2;
  const double inv = fast_rcp(6.0 * (dl * dr));
  fl = c + nl * (dr * inv);
  fr = c + nr * (dl * inv);
}

// FP32 WENO5-Z: products of s's would overflow float for pressure-sized data,
// so each weight uses a hardware reciprocal of its s_k and each biased value
// its own normalization.
__device__ __forceinline__ void weno5_z(float a, float b, float c, float d, float e, float eps, float& fl,
                                        float& fr) {
  const float D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const float u0 = D1 - D0, v0 = 3.0f * D1 - D0;
  const float u1 = D2 - D1, v1 = D1 + D2;
  const float u2 = D3 - D2, v2 = D3 - 3.0f * D2;
  const float e4 = 4.0f * eps;
  const float s0 = e4 + ((13.0f / 3.0f) * u0 * u0 + v0 * v0);
  const float s1 = e4 + ((13.0f / 3.0f) * u1 * u1 + v1 * v1);
  const float s2 = e4 + ((13.0f / 3.0f) * u2 * u2 + v2 * v2);
  const float tau = fabsf(s0 - s2);
  const float g0 = 1.0f + tau * __builtin_amdgcn_rcpf(s0);
  const float g1 = 1.0f + tau * __builtin_amdgcn_rcpf(s1);
  const float g2 = 1.0f + tau * __builtin_amdgcn_rcpf(s2);
  const float l0 = 5.0f * D1 - 2.0f * D0, l1 = D1 + 2.0f * D2, l2 = 4.0f * D2 - D3;
  const float r0 = 2.0f * D3 - 5.0f * D2, r1 = -(D2 + 2.0f * D1), r2 = D0 - 4.0f * D1;
  const float w1 = 0.6f * g1;
  const float wl0 = 0.1f * g0, wl2 = 0.3f * g2;
  const float wr0 = 0.1f * g2, wr2 = 0.3f * g0;
  fl = c + (wl0 * l0 + w1 * l1 + wl2 * l2) * __builtin_amdgcn_rcpf(6.0f * (wl0 + w1 + wl2));
  fr = c + (wr0 * r0 + w1 * r1 + wr2 * r2) * __builtin_amdgcn_rcpf(6.0f * (wr0 + w1 + wr2));
}

// TENO5 (Sec. 4.2.2): the same candidates and indicators; stencil k is kept
// when its share of gamma_k = d_k (1 + tau/(beta_k + eps))^6 reaches the
// cut-off kTenoCt, and the kept stencils combine with their linear weights.
// In terms of s_k = 4 (eps + beta_k): 1 + tau/(beta_k + eps) = 1 + tau'/s_k
// with tau' = |s_0 - s_2|.  The shares are compared as gamma_k >= C_T sum gamma.
constexpr double kTenoCt = 1e-5;

__host__ __device__ __forceinline__ void teno5(double a, double b, double c, double d, double e, double eps,
                                               double& fl, double& fr) {
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
  const double p0 = (x0 * x0) * (x0 * x0) * (x0 * x0);
  const double p1 = (x1 * x1) * (x1 * x1) * (x1 * x1);
  const double p2 = (x2 * x2) * (x2 * x2) * (x2 * x2);
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double r0 = 2.0 * D3 - 5.0 * D2, r1 = -(D2 + 2.0 * D1), r2 = D0 - 4.0 * D1;
  // left: linear weights (0.1, 0.6, 0.3) on stencils (0, 1, 2); right: mirrored
  const double gl0 = 0.1 * p0, g1 = 0.6 * p1, gl2 = 0.3 * p2;
  const double gr0 = 0.1 * p2, gr2 = 0.3 * p0;
  const double cl = kTenoCt * (gl0 + g1 + gl2), cr = kTenoCt * (gr0 + g1 + gr2);
  const double wl0 = gl0 >= cl ? 0.1 : 0.0, wl1 = g1 >= cl ? 0.6 : 0.0, wl2 = gl2 >= cl ? 0.3 : 0.0;
  const double wr0 = gr0 >= cr ? 0.1 : 0.0, wr1 = g1 >= cr ? 0.6 : 0.0, wr2 = gr2 >= cr ? 0.3 : 0.0;
  const double inv = fast_rcp(6.0 * ((wl0 + wl1 + wl2) * (wr0 + wr1 + wr2)));
  fl = c + (wl0 * l0 + wl1 * l1 + wl2 * l2) * ((wr0 + wr1 + wr2) * inv);
  fr = c + (wr0 * r0 + wr1 * r1 + wr2 * r2) * ((wl0 + wl1 + wl2) * inv);
}

// FP32 TENO5: x_k = 1 + tau'/s_k is scaled by its maximum before the sixth
// power (which would overflow float); the shares are unchanged by the scale.
__device__ __forceinline__ void teno5(float a, float b, float c, float d, float e, float eps, float& fl,
                                      float& fr) {
  const float D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const float u0 = D1 - D0, v0 = 3.0f * D1 - D0;
  const float u1 = D2 - D1, v1 = D1 + D2;
  const float u2 = D3 - D2, v2 = D3 - 3.0f * D2;
  const float e4 = 4.0f * eps;
  const float s0 = e4 + ((13.0f / 3.0f) * u0 * u0 + v0 * v0);
  const float s1 = e4 + ((13.0f / 3.0f) * u1 * u1 + v1 * v1);
  const float s2 = e4 + ((13.0f / 3.0f) * u2 * u2 + v2 * v2);
  const float tau = fabsf(s0 - s2);
  float x0 = 1.0f + tau * __builtin_amdgcn_rcpf(s0);
  float x1 = 1.0f + tau * __builtin_amdgcn_rcpf(s1);
  float x2 = 1.0f + tau * __builtin_amdgcn_rcpf(s2);
  const float xm = __builtin_amdgcn_rcpf(fmaxf(x0, fmaxf(x1, x2)));
  x0 *= xm;
  x1 *= xm;
  x2 *= xm;
  const float p0 = (x0 * x0) * (x0 * x0) * (x0 * x0);
  const float p1 = (x1 * x1) * (x1 * x1) * (x1 * x1);
  const float p2 = (x2 * x2) * (x2 * x2) * (x2 * x2);
  const float l0 = 5.0f * D1 - 2.0f * D0, l1 = D1 + 2.0f * D2, l2 = 4.0f * D2 - D3;
  const float r0 = 2.0f * D3 - 5.0f * D2, r1 = -(D2 + 2.0f * D1), r2 = D0 - 4.0f * D1;
  const float gl0 = 0.1f * p0, g1 = 0.6f * p1, gl2 = 0.3f * p2;
  const float gr0 = 0.1f * p2, gr2 = 0.3f * p0;
  const float ct = float(kTenoCt);
  const float cl = ct * (gl0 + g1 + gl2), cr = ct * (gr0 + g1 + gr2);
  const float wl0 = gl0 >= cl ? 0.1f : 0.0f, wl1 = g1 >= cl ? 0.6f : 0.0f, wl2 = gl2 >= cl ? 0.3f : 0.0f;
  const float wr0 = gr0 >= cr ? 0.1f : 0.0f, wr1 = g1 >= cr ? 0.6f : 0.0f, wr2 = gr2 >= cr ? 0.3f : 0.0f;
  fl = c + (wl0 * l0 + wl1 * l1 + wl2 * l2) * __builtin_amdgcn_rcpf(6.0f * (wl0 + wl1 + wl2));
  fr = c + (wr0 * r0 + wr1 * r1 + wr2 * r2) * __builtin_amdgcn_rcpf(6.0f * (wr0 + wr1 + wr2));
}

// WENO5-M (Sec. 3.2.1: fifth order kept by the mapped weights of Henrick,
// Aslam and Powers).  The JS weights w_k of weno5_js, normalized, are mapped by
//   g_k(w) = w (d_k + d_k^2 - 3 d_k w + w^2) / (d_k^2 + w (1 - 2 d_k))
// and normalized again.  Mapped weight k is N_k/Q_k with Q_k >= d_k min(d_k,
// 1 - d_k) > 0 on [0, 1]; over the common denominator Q_0 Q_1 Q_2 each side's
// normalization is one sum, so one refined reciprocal serves the JS
// normalization of both sides and one the mapped normalization of both.
__host__ __device__ __forceinline__ void weno_m_map(double w, double dk, double& num, double& den) {
  num = w * ((dk + dk * dk) + w * (w - 3.0 * dk));
  den = dk * dk + w * (1.0 - 2.0 * dk);
}

__host__ __device__ __forceinline__ void weno5_m(double a, double b, double c, double d, double e, double eps,
                                                 double& fl, double& fr) {
  const double D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const double u0 = D1 - D0, v0 = 3.0 * D1 - D0;
  const double u1 = D2 - D1, v1 = D1 + D2;
  const double u2 = D3 - D2, v2 = D3 - 3.0 * D2;
  const double e4 = 4.0 * eps;
  const double s0 = e4 + ((13.0 / 3.0) * u0 * u0 + v0 * v0);
  const double s1 = e4 + ((13.0 / 3.0) * u1 * u1 + v1 * v1);
  const double s2 = e4 + ((13.0 / 3.0) * u2 * u2 + v2 * v2);
  const double t0 = s0 * s0, t1 = s1 * s1, t2 = s2 * s2;
  const double p0 = t1 * t2, p1 = t0 * t2, p2 = t0 * t1;
  const double w1 = 0.6 * p1;
  const double wl0 = 0.1 * p0, wl2 = 0.3 * p2;
  const double wr0 = 0.1 * p2, wr2 = 0.3 * p0;
  const double dl = wl0 + w1 + wl2;
  const double dr = wr0 + w1 + wr2;
  const double inv = fast_rcp(dl * dr);
  const double idl = dr * inv, idr = dl * inv;
  // left: d = (0.1, 0.6, 0.3) on candidates l0, l1, l2; right: the mirror
  double nl0, ql0, nl1, ql1, nl2, ql2, nr0, qr0, nr1, qr1, nr2, qr2;
  weno_m_map(wl0 * idl, 0.1, nl0, ql0);
  weno_m_map(w1 * idl, 0.6, nl1, ql1);
  weno_m_map(wl2 * idl, 0.3, nl2, ql2);
  weno_m_map(wr0 * idr, 0.1, nr0, qr0);
  weno_m_map(w1 * idr, 0.6, nr1, qr1);
  weno_m_map(wr2 * idr, 0.3, nr2, qr2);
  const double el0 = nl0 * (ql1 * ql2), el1 = nl1 * (ql0 * ql2), el2 = nl2 * (ql0 * ql1);
  const double er0 = nr0 * (qr1 * qr2), er1 = nr1 * (qr0 * qr2), er2 = nr2 * (qr0 * qr1);
  const double hl = el0 + el1 + el2, hr = er0 + er1 + er2;
  const double l0 = 5.0 * D1 - 2.0 * D0, l1 = D1 + 2.0 * D2, l2 = 4.0 * D2 - D3;
  const double r0 = 2.0 * D3 - 5.0 * D2, r1 = -(D2 + 2.0 * D1), r2 = D0 - 4.0 * D1;
  const double inv2 = fast_rcp(6.0 * (hl * hr));
  fl = c + (el0 * l0 + el1 * l1 + el2 * l2) * (hr * inv2);
  fr = c + (er0 * r0 + er1 * r1 + er2 * r2) * (hl * inv2);
}

// FP32 WENO5-M: the JS weights of the float weno5_js (ratios s_min/s_k, so
// that nothing overflows), normalized, mapped in float and normalized per side.
__device__ __forceinline__ void weno5_m(float a, float b, float c, float d, float e, float eps, float& fl,
                                        float& fr) {
  const float D0 = b - a, D1 = c - b, D2 = d - c, D3 = e - d;
  const float u0 = D1 - D0, v0 = 3.0f * D1 - D0;
  const float u1 = D2 - D1, v1 = D1 + D2;
  const float u2 = D3 - D2, v2 = D3 - 3.0f * D2;
  const float e4 = 4.0f * eps;
  const float s0 = e4 + ((13.0f / 3.0f) * u0 * u0 + v0 * v0);
  const float s1 = e4 + ((13.0f / 3.0f) * u1 * u1 + v1 * v1);
  const float s2 = e4 + ((13.0f / 3.0f) * u2 * u2 + v2 * v2);
  const float sm = fminf(s0, fminf(s1, s2));
  const float a0 = sq(sm * __builtin_amdgcn_rcpf(s0));
  const float a1 = sq(sm * __builtin_amdgcn_rcpf(s1));
  const float a2 = sq(sm * __builtin_amdgcn_rcpf(s2));
  const float w1 = 0.6f * a1;
  const float wl0 = 0.1f * a0, wl2 = 0.3f * a2;
  const float wr0 = 0.1f * a2, wr2 = 0.3f * a0;
  const float idl = __builtin_amdgcn_rcpf(wl0 + w1 + wl2);
  const float idr = __builtin_amdgcn_rcpf(wr0 + w1 + wr2);
  auto map = [](float w, float dk, float& num, float& den) {
    num = w * ((dk + dk * dk) + w * (w - 3.0f * dk));
    den = dk * dk + w * (1.0f - 2.0f * dk);
  };
  float nl0, ql0, nl1, ql1, nl2, ql2, nr0, qr0, nr1, qr1, nr2, qr2;
  map(wl0 * idl, 0.1f, nl0, ql0);
  map(w1 * idl, 0.6f, nl1, ql1);
  map(wl2 * idl, 0.3f, nl2, ql2);
  map(wr0 * idr, 0.1f, nr0, qr0);
  map(w1 * idr, 0.6f, nr1, qr1);
  map(wr2 * idr, 0.3f, nr2, qr2);
  const float el0 = nl0 * (ql1 * ql2), el1 = nl1 * (ql0 * ql2), el2 = nl2 * (ql0 * ql1);
  const float er0 = nr0 * (qr1 * qr2), er1 = nr1 * (qr0 * qr2), er2 = nr2 * (qr0 * qr1);
  const float l0 = 5.0f * D1 - 2.0f * D0, l1 = D1 + 2.0f * D2, l2 = 4.0f * D2 - D3;
  const float r0 = 2.0f * D3 - 5.0f * D2, r1 = -(D2 + 2.0f * D1), r2 = D0 - 4.0f * D1;
  fl = c + (el0 * l0 + el1 * l1 + el2 * l2) * __builtin_amdgcn_rcpf(6.0f * (el0 + el1 + el2));
  fr = c + (er0 * r0 + er1 * r1 + er2 * r2) * __builtin_amdgcn_rcpf(6.0f * (er0 + er1 + er2));
}

// ---------------------------------------------------------------------------
// WENO5-JS on a non-uniform grid (Sec. 4.2.2): the candidates and smoothness
// indicators of the centre's tabulated quadratics and the grid's ideal weights.
// In the unit coordinate of the centre cell the candidate values at the right
// and left faces are f_2 + m0' +- m1/2 + m2/4 (m0' = m0 - f_2) and the
// indicator sum_{l=1,2} h^(2l-1) int (d^l p/dx^l)^2 dx is m1^2 + (13/3) m2^2.
// `cf` points at the centre's entry of row 0 and `st` is the row stride.
// fr: value at the right face (left state of the face c + 1/2); fl: value at
// the left face (right state of the face c - 1/2).
// ---------------------------------------------------------------------------
template <typename T, typename C>
__device__ __forceinline__ void nu_candidates(const T* D, const C* cf, long long st, T* qr, T* ql, T* beta) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T da = D[r], db = D[r + 1];
    const T mu0 = T(cf[(NU_MU0 + 2 * r) * st]) * da + T(cf[(NU_MU0 + 2 * r + 1) * st]) * db;
    const T m1 = T(cf[(NU_M1 + 2 * r) * st]) * da + T(cf[(NU_M1 + 2 * r + 1) * st]) * db;
    const T m2 = T(cf[(NU_M2 + 2 * r) * st]) * da + T(cf[(NU_M2 + 2 * r + 1) * st]) * db;
    const T even = mu0 + T(0.25) * m2;
    qr[r] = even + T(0.5) * m1;
    ql[r] = even - T(0.5) * m1;
    beta[r] = m1 * m1 + T(13.0 / 3.0) * (m2 * m2);
  }
}

// Double: the weights d_r/(eps + beta_r)^2 over the common denominator
// t0 t1 t2, both normalizations from one refined reciprocal (as weno5_js).
__device__ __forceinline__ void weno5_nu(double a, double b, double c, double d, double e, double eps,
                                         const double* cf, long long st, double& fr, double& fl) {
  const double D[4] = {b - a, c - b, d - c, e - d};
  double qr[3], ql[3], beta[3];
  nu_candidates<double, double>(D, cf, st, qr, ql, beta);
  const double t0 = sq(eps + beta[0]), t1 = sq(eps + beta[1]), t2 = sq(eps + beta[2]);
  const double p0 = t1 * t2, p1 = t0 * t2, p2 = t0 * t1;
  const double wr0 = cf[(NU_DR + 0) * st] * p0, wr1 = cf[(NU_DR + 1) * st] * p1, wr2 = cf[(NU_DR + 2) * st] * p2;
  const double wl0 = cf[(NU_DL + 0) * st] * p0, wl1 = cf[(NU_DL + 1) * st] * p1, wl2 = cf[(NU_DL + 2) * st] * p2;
  const double sr = wr0 + wr1 + wr2, sl = wl0 + wl1 + wl2;
  const double inv = fast_rcp(sr * sl);
  fr = c + (wr0 * qr[0] + wr1 * qr[1] + wr2 * qr[2]) * (sl * inv);
  fl = c + (wl0 * ql[0] + wl1 * ql[1] + wl2 * ql[2]) * (sr * inv);
}

// Float: the weights from the ratios s_min/s_r, s_r = eps + beta_r (as the
// float weno5_js), each side normalized on its own.
__device__ __forceinline__ void weno5_nu(float a, float b, float c, float d, float e, float eps, const float* cf,
                                         long long st, float& fr, float& fl) {
  const float D[4] = {b - a, c - b, d - c, e - d};
  float qr[3], ql[3], beta[3];
  nu_candidates<float, float>(D, cf, st, qr, ql, beta);
  const float s0 = eps + beta[0], s1 = eps + beta[1], s2 = eps + beta[2];
  const float sm = fminf(s0, fminf(s1, s2));
  const float a0 = sq(sm * __builtin_amdgcn_rcpf(s0));
  const float a1 = sq(sm * __builtin_amdgcn_rcpf(s1));
  const float a2 = sq(sm * __builtin_amdgcn_rcpf(s2));
  const float wr0 = cf[(NU_DR + 0) * st] * a0, wr1 = cf[(NU_DR + 1) * st] * a1, wr2 = cf[(NU_DR + 2) * st] * a2;
  const float wl0 = cf[(NU_DL + 0) * st] * a0, wl1 = cf[(NU_DL + 1) * st] * a1, wl2 = cf[(NU_DL + 2) * st] * a2;
  fr = c + (wr0 * qr[0] + wr1 * qr[1] + wr2 * qr[2]) * __builtin_amdgcn_rcpf(wr0 + wr1 + wr2);
  fl = c + (wl0 * ql[0] + wl1 * ql[1] + wl2 * ql[2]) * __builtin_amdgcn_rcpf(wl0 + wl1 + wl2);
}

// Maximum over the 64 lanes of a wave (NaN-ignoring, as fmax).
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Signal speed of one cell for the CFL step: sum_d (|u_d| + c)/dx_d from the
// conservative U and primitive W of the cell (c: frozen-mixture sound speed).
// bad: c^2 <= 0 or a non-finite result.
template <int NF, int D>
__device__ __forceinline__ double cell_signal(const Params& pm, const double* U, const double* W, bool& bad,
                                              const double* inv_h) {
  using R = Rows<NF, D>;
  double rho = U[0];
  if constexpr (NF == 2) rho = U[0] + U[1];
  double Gam, Pi;
  if constexpr (NF == 2)
    mixture<NF, double>(pm, U[R::ALPHA], U[R::ALPHA + 1], Gam, Pi);
  else
    mixture<NF, double>(pm, 1.0, 0.0, Gam, Pi);
  const double c2 = sound_speed_sq(rho, W[R::E], Gam, Pi);
  const double cs = sqrt(c2);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) s += (fabs(W[R::MOM + d]) + cs) * inv_h[d];
  bad = !(c2 > 0.0) || !isfinite(s);
  return s;
}

// The reconstruction of a kernel instantiation: WV = 0 WENO5-JS, 1 WENO5-Z,
// 2 TENO5, 3 WENO5-M.  (A compile-time choice: a run-time branch inside the unrolled row
// loops would make every kernel hold the registers of all of them.)
template <int WV, typename T>
__device__ __forceinline__ void weno5(T a, T b, T c, T d, T e, T eps, T& fl, T& fr) {
  if constexpr (WV == 1)
    weno5_z(a, b, c, d, e, eps, fl, fr);
  else if constexpr (WV == 2)
    teno5(a, b, c, d, e, eps, fl, fr);
  else if constexpr (WV == 3)
    weno5_m(a, b, c, d, e, eps, fl, fr);
  else
    weno5_js(a, b, c, d, e, eps, fl, fr);
}

// ---------------------------------------------------------------------------
// HLLC face solver (Sec. 3.2.2; star states of Toro's book), returning the flux
// of every row and the face velocity u_f.  T is the flux arithmetic type;
// sound speeds and the wave speeds S_L, S_R, S* are always double.
//   S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R) (the form
//   printed for the HLLD solver, Sec. 4.2.5), ties to the first argument;
//   regions: S_L >= 0 left; S* >= 0 left star; S_R > 0 right star; else right;
//   volume fractions are carried by the contact: flux alpha_K u_f.
// Returns true when a side has c^2 <= 0 or a flux is not finite.
// ---------------------------------------------------------------------------
template <int NF, int D, int DIR, typename T, bool APC = false>
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
  // the denominator is strictly negative for physical states (S_L < u_L, S_R > u_R)
  const double rden = fast_rcp(drhoR * (SR - dunR) - drhoL * (SL - dunL));
  const double Sstar = (double(pR) - double(pL) + drhoL * dunL * (SL - dunL) - drhoR * dunR * (SR - dunR)) * -rden;

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
  const double chi = star ? skmu * fast_rcp(SK - Sstar) : 1.0;
  const double p_over = double(p) * fast_rcp(skmu);
  const T s = star ? T(SK) : T(0);
  const T chiT = T(chi);
  const T SstarT = T(Sstar);
  // anti-dissipation pressure correction of Chen et al. (Sec. 4.2.4) on both
  // star fluxes: (z - 1) p_d on the normal momentum and (z - 1) p_d S* on the
  // energy, with p_d = rho_L rho_R (S_L - u_L)(S_R - u_R)(u_R - u_L) /
  // (rho_R (S_R - u_R) - rho_L (S_L - u_L)) (the velocity-jump part of the star
  // pressure) and z = min(max(|u_L|/c_L, |u_R|/c_R), 1); double arithmetic
  T apc_m = T(0), apc_e = T(0);
  if constexpr (APC) {
    const double mL = fabs(dunL) * fast_rcp(cL), mR = fabs(dunR) * fast_rcp(cR);
    double z = (mL >= mR) ? mL : mR;
    if (z > 1.0) z = 1.0;
    const double pd = drhoL * drhoR * (SL - dunL) * (SR - dunR) * (dunR - dunL) * rden;
    const double am = star ? (z - 1.0) * pd : 0.0;
    apc_m = T(am);
    apc_e = T(am * Sstar);
  }
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
    const T Es = chiT * (E + (SstarT - un) * (rho * SstarT + T(p_over)));
    F[R::E] = (E + p) * un + s * (Es - E);
  }
  if constexpr (APC) {
    F[R::MOM + DIR] = F[R::MOM + DIR] + apc_m;
    F[R::E] = F[R::E] + apc_e;
  }
  uf = star ? SstarT : un;
  if constexpr (NF == 2) {
    F[R::ALPHA] = W[R::ALPHA] * uf;
    F[R::ALPHA + 1] = W[R::ALPHA + 1] * uf;
  }
  // explicit class checks: an "x - x == 0" test would not survive fused
  // multiply-add contraction (a*b - a*b becomes the rounding residual)
  bool finite = __builtin_isfinite(uf);
#pragma unroll
  for (int v = 0; v < R::NEQ; ++v) finite = finite && __builtin_isfinite(F[v]);
  return !(c2L > 0.0 && c2R > 0.0 && finite);
}

// ---------------------------------------------------------------------------
// HLL face solver (Sec. 3.2.2; Toro's book): two waves, the HLLC estimates
// S_L, S_R, and one averaged state between them.  Per face the flux is
//   F = (a F_L + b F_R + c (U_R - U_L)) r
// with (a, b, c, r) = (1, 0, 0, 1) for S_L >= 0, (0, 1, 0, 1) for S_R <= 0,
// and (S_R, -S_L, S_L S_R, 1/(S_R - S_L)) otherwise; every row's U and F are
// formed from the side's primitives as they are used.  Volume fractions take
// the same formula on alpha u_n, and the face velocity is (a u_L + b u_R) r,
// so that a uniform alpha stays uniform.  Returns true as hllc does.
// ---------------------------------------------------------------------------
template <int NF, int D, int DIR, typename T>
__host__ __device__ __forceinline__ bool hll(const Params& pm, const T* WL, const T* WR, T* F, T& uf) {
  using R = Rows<NF, D>;
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
  double a, b, c, r;
  if (SL >= 0.0) {
    a = 1.0;
    b = 0.0;
    c = 0.0;
    r = 1.0;
  } else if (SR <= 0.0) {
    a = 0.0;
    b = 1.0;
    c = 0.0;
    r = 1.0;
  } else {
    a = SR;
    b = -SL;
    c = SL * SR;
    r = fast_rcp(SR - SL);
  }
  const T aT = T(a), bT = T(b), cT = T(c), rT = T(r);
  T usqL = T(0), usqR = T(0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    usqL += WL[R::MOM + e] * WL[R::MOM + e];
    usqR += WR[R::MOM + e] * WR[R::MOM + e];
  }
  const T EL = GamL * pL + PiL + T(0.5) * rhoL * usqL;
  const T ER = GamR * pR + PiR + T(0.5) * rhoR * usqR;
#pragma unroll
  for (int i = 0; i < NF; ++i) F[i] = (aT * (WL[i] * unL) + bT * (WR[i] * unR) + cT * (WR[i] - WL[i])) * rT;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    const T mL = rhoL * WL[R::MOM + e], mR = rhoR * WR[R::MOM + e];
    const T fL = mL * unL + ((e == DIR) ? pL : T(0));
    const T fR = mR * unR + ((e == DIR) ? pR : T(0));
    F[R::MOM + e] = (aT * fL + bT * fR + cT * (mR - mL)) * rT;
  }
  F[R::E] = (aT * ((EL + pL) * unL) + bT * ((ER + pR) * unR) + cT * (ER - EL)) * rT;
  uf = (aT * unL + bT * unR) * rT;
  if constexpr (NF == 2) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T aL = WL[R::ALPHA + k], aR = WR[R::ALPHA + k];
      F[R::ALPHA + k] = (aT * (aL * unL) + bT * (aR * unR) + cT * (aR - aL)) * rT;
    }
  }
  bool finite = __builtin_isfinite(uf);
#pragma unroll
  for (int v = 0; v < R::NEQ; ++v) finite = finite && __builtin_isfinite(F[v]);
  return !(c2L > 0.0 && c2R > 0.0 && finite);
}

// Low-Mach correction of Thornber et al. (the paper's low-Mach section): with
// z = min(max(|u_L|/c_L, |u_R|/c_R), 1), sound speeds of the states as
// reconstructed, the face-normal velocities become
//   u_L* = (u_L + u_R)/2 + z (u_L - u_R)/2,  u_R* = (u_L + u_R)/2 + z (u_R - u_L)/2
// and replace u_L, u_R in the face solver.  The Mach numbers and z in double.
template <int NF, int D, int DIR, typename T>
__host__ __device__ __forceinline__ void thornber(const Params& pm, T* WL, T* WR) {
  using R = Rows<NF, D>;
  double rhoL = double(WL[0]), rhoR = double(WR[0]);
  if constexpr (NF == 2) {
    rhoL = double(WL[0]) + double(WL[1]);
    rhoR = double(WR[0]) + double(WR[1]);
  }
  double GamL, PiL, GamR, PiR;
  if constexpr (NF == 2) {
    mixture<NF, double>(pm, double(WL[R::ALPHA]), double(WL[R::ALPHA + 1]), GamL, PiL);
    mixture<NF, double>(pm, double(WR[R::ALPHA]), double(WR[R::ALPHA + 1]), GamR, PiR);
  } else {
    mixture<NF, double>(pm, 1.0, 0.0, GamL, PiL);
    mixture<NF, double>(pm, 1.0, 0.0, GamR, PiR);
  }
  const double uL = double(WL[R::MOM + DIR]), uR = double(WR[R::MOM + DIR]);
  const double cL = sqrt(sound_speed_sq(rhoL, double(WL[R::E]), GamL, PiL));
  const double cR = sqrt(sound_speed_sq(rhoR, double(WR[R::E]), GamR, PiR));
  const double mL = fabs(uL) / cL, mR = fabs(uR) / cR;
  double z = (mL >= mR) ? mL : mR;
  if (z > 1.0) z = 1.0;
  WL[R::MOM + DIR] = T(0.5 * (uL + uR) + z * (0.5 * (uL - uR)));
  WR[R::MOM + DIR] = T(0.5 * (uL + uR) + z * (0.5 * (uR - uL)));
}

// Compile-time face options of a kernel instantiation (bits of RS).
enum { RS_HLL = 1, RS_THORNBER = 2, RS_APC = 4, RS_KAPILA = 8 };

// The face solver of a kernel instantiation: HLL when RS has RS_HLL, else
// HLLC, with the APC term when RS has RS_APC.
template <int RS, int NF, int D, int DIR, typename T>
__host__ __device__ __forceinline__ bool riemann(const Params& pm, const T* WL, const T* WR, T* F, T& uf) {
  if constexpr ((RS & RS_HLL) != 0)
    return hll<NF, D, DIR, T>(pm, WL, WR, F, uf);
  else
    return hllc<NF, D, DIR, T, (RS & RS_APC) != 0>(pm, WL, WR, F, uf);
}

}  // namespace mfc
