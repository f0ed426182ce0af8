/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the five-equation (Allaire)
 * right-hand side with stiffened-gas closure, WENO5-JS reconstruction of
 * primitive variables, HLLC face fluxes and SSP-RK3 time stepping.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP library and the HIP library never calls it.
 *
 * Every routine follows the paper (arXiv 2503.07953, "MFC 5.0") in its own
 * order and notation; where the paper is silent the reading used is stated
 * next to the code.  Built with -O2 -ffp-contract=off (no fused multiply-add,
 * no fast-math), OpenMP only across independent grid lines or cells.
 *
 * State layout: q[v][k][j][i], x fastest, interior cells only, float64.
 * Rows for nf fluids in D dimensions (Sec. 2.1.1, eq. five_eqn_transport):
 *   alpha_i rho_i (nf rows), rho u_d (D rows), rho E, alpha_i (nf rows, only
 *   when nf == 2; a single fluid is the Euler system and carries none).
 * Primitive rows: alpha_i rho_i, u_d, p, alpha_i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NONFINITE (-5)

#define BC_PERIODIC 0
#define BC_EXTRAP 1
#define BC_SLIPWALL 2

#define NEQ_MAX 8

/* TENO5 cut-off C_T (not printed in the paper; the value published with the
 * fifth-order TENO construction). */
#define ORC_TENO_CT 1e-5

typedef struct {
  int32_t ndim;
  int32_t n[3];
  int32_t num_fluids;
  int32_t bc_lo[3], bc_hi[3];
  double dx[3];
  double gamma[2], pi_inf[2];
  double weno_eps;
  int32_t weno_variant; /* 0: WENO5-JS (Sec. 3.2.1), 1: WENO5-Z, 2: TENO5 (Sec. 4.2.2), 3: WENO5-M (Sec. 3.2.1) */
  int32_t riemann;      /* 0: HLLC, 1: HLL (Sec. 3.2.2) */
  int32_t low_mach;     /* 0: none, 1: the Thornber et al. velocity correction, 2: the anti-dissipation
                           pressure correction of Chen et al. (HLLC only) (Sec. 4.2.4) */
  int32_t model;        /* 0: Allaire (K = 0), 1: Kapila, K div u on the alpha rows (Sec. 2.1.1) */
  const double* faces[3]; /* per axis: NULL (uniform spacing dx) or the n + 1 cell-face coordinates of a
                             non-uniform grid, strictly increasing (Sec. 4.2.2); WENO5-JS only */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Row bookkeeping                                                          */
/* ------------------------------------------------------------------------ */
int orc_num_eqs(const orc_problem* P) {
  int nf = P->num_fluids, D = P->ndim;
  return nf + D + 1 + (nf == 2 ? 2 : 0);
}
static int row_mom(const orc_problem* P, int d) { return P->num_fluids + d; }
static int row_E(const orc_problem* P) { return P->num_fluids + P->ndim; }
static int row_alpha(const orc_problem* P, int i) { return P->num_fluids + P->ndim + 1 + i; }
static int64_t ncell(const orc_problem* P) {
  return (int64_t)P->n[0] * P->n[1] * P->n[2];
}

int orc_validate(const orc_problem* P) {
  if (!P) return ORC_ERR_ARG;
  if (P->ndim < 1 || P->ndim > 3) return ORC_ERR_ARG;
  if (P->num_fluids != 1 && P->num_fluids != 2) return ORC_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    if (d < P->ndim) {
      if (P->n[d] < 3) return ORC_ERR_ARG;
      if (!(P->dx[d] > 0)) return ORC_ERR_ARG;
      if ((P->bc_lo[d] == BC_PERIODIC) != (P->bc_hi[d] == BC_PERIODIC)) return ORC_ERR_ARG;
      if (P->bc_lo[d] < 0 || P->bc_lo[d] > 2 || P->bc_hi[d] < 0 || P->bc_hi[d] > 2)
        return ORC_ERR_ARG;
    } else if (P->n[d] != 1) {
      return ORC_ERR_ARG;
    }
  }
  for (int i = 0; i < P->num_fluids; ++i)
    if (!(P->gamma[i] > 1.0) || !(P->pi_inf[i] >= 0.0)) return ORC_ERR_ARG;
  if (!(P->weno_eps > 0)) return ORC_ERR_ARG;
  if (P->weno_variant < 0 || P->weno_variant > 3) return ORC_ERR_ARG;
  if (P->riemann < 0 || P->riemann > 1) return ORC_ERR_ARG;
  if (P->low_mach < 0 || P->low_mach > 2) return ORC_ERR_ARG;
  if (P->low_mach == 2 && P->riemann != 0) return ORC_ERR_ARG;
  if (P->model < 0 || P->model > 1) return ORC_ERR_ARG;
  if (P->model == 1 && P->num_fluids != 2) return ORC_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    if (!P->faces[d]) continue;
    if (d >= P->ndim || P->weno_variant != 0) return ORC_ERR_ARG;
    for (int i = 0; i < P->n[d]; ++i)
      if (!(P->faces[d][i + 1] > P->faces[d][i]) || !isfinite(P->faces[d][i + 1] - P->faces[d][i]))
        return ORC_ERR_ARG;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Stiffened-gas mixture closure (Sec. 2.1.1 mixture rules, Sec. 2.2 eq. eos) */
/*   rho_i e_i = (p + gamma_i pi_i)/(gamma_i - 1) = p G_i + P_i with         */
/*   G_i = 1/(gamma_i - 1), P_i = gamma_i pi_i/(gamma_i - 1); so the mixture */
/*   rho e = sum alpha_i rho_i e_i = Gamma p + Pi with Gamma = sum alpha_i   */
/*   G_i and Pi = sum alpha_i P_i.  A single fluid has alpha = 1.            */
/* ------------------------------------------------------------------------ */
static double fluid_G(const orc_problem* P, int i) { return 1.0 / (P->gamma[i] - 1.0); }
static double fluid_P(const orc_problem* P, int i) {
  return P->gamma[i] * P->pi_inf[i] / (P->gamma[i] - 1.0);
}

static void mixture(const orc_problem* P, const double* alpha, double* Gam, double* Pi) {
  if (P->num_fluids == 1) {
    *Gam = fluid_G(P, 0);
    *Pi = fluid_P(P, 0);
    return;
  }
  *Gam = alpha[0] * fluid_G(P, 0) + alpha[1] * fluid_G(P, 1);
  *Pi = alpha[0] * fluid_P(P, 0) + alpha[1] * fluid_P(P, 1);
}

/* conservative -> primitive for one cell: u_d = (rho u_d)/rho,
 * p = (rho E - rho|u|^2/2 - Pi)/Gamma. */
static void cell_cons_to_prim(const orc_problem* P, const double* U, double* W) {
  int nf = P->num_fluids, D = P->ndim, neq = orc_num_eqs(P);
  double rho = 0.0;
  for (int i = 0; i < nf; ++i) rho = rho + U[i];
  double usq = 0.0;
  for (int d = 0; d < D; ++d) {
    double u = U[row_mom(P, d)] / rho;
    W[row_mom(P, d)] = u;
    usq = usq + u * u;
  }
  double Gam, Pi;
  mixture(P, nf == 2 ? &U[row_alpha(P, 0)] : NULL, &Gam, &Pi);
  double ke = 0.5 * rho * usq;
  W[row_E(P)] = (U[row_E(P)] - ke - Pi) / Gam;
  for (int i = 0; i < nf; ++i) W[i] = U[i];
  for (int v = row_E(P) + 1; v < neq; ++v) W[v] = U[v];
}

/* primitive -> conservative for one cell: rho E = Gamma p + Pi + rho|u|^2/2. */
static void cell_prim_to_cons(const orc_problem* P, const double* W, double* U) {
  int nf = P->num_fluids, D = P->ndim, neq = orc_num_eqs(P);
  double rho = 0.0;
  for (int i = 0; i < nf; ++i) rho = rho + W[i];
  double usq = 0.0;
  for (int d = 0; d < D; ++d) {
    double u = W[row_mom(P, d)];
    U[row_mom(P, d)] = rho * u;
    usq = usq + u * u;
  }
  double Gam, Pi;
  mixture(P, nf == 2 ? &W[row_alpha(P, 0)] : NULL, &Gam, &Pi);
  double ke = 0.5 * rho * usq;
  U[row_E(P)] = Gam * W[row_E(P)] + Pi + ke;
  for (int i = 0; i < nf; ++i) U[i] = W[i];
  for (int v = row_E(P) + 1; v < neq; ++v) U[v] = W[v];
}

/* Squared sound speed of the mixture read as one stiffened gas with
 * gamma_m = 1 + 1/Gamma and pi_m = Pi/(Gamma + 1):
 * c^2 = gamma_m (p + pi_m)/rho = ((Gamma + 1) p + Pi)/(Gamma rho).
 * For a pure fluid this is gamma_i (p + pi_i)/rho_i (Sec. 2.1.1). */
static double sound_speed_sq(double rho, double p, double Gam, double Pi) {
  return ((Gam + 1.0) * p + Pi) / (Gam * rho);
}

/* ------------------------------------------------------------------------ */
/* Ghost layers (Sec. 3.3): three buffer cells per side per axis.           */
/*   periodic: wrap; extrapolation: copy of the nearest interior cell       */
/*   (zeroth degree); slip wall: mirror image with the wall-normal          */
/*   momentum negated.                                                      */
/* ------------------------------------------------------------------------ */
static int ghost_map(const orc_problem* P, int d, int g, int* flip) {
  int n = P->n[d];
  if (g < 0) {
    switch (P->bc_lo[d]) {
      case BC_PERIODIC: return g + n;
      case BC_EXTRAP: return 0;
      default: *flip = 1; return -1 - g;
    }
  }
  if (g >= n) {
    switch (P->bc_hi[d]) {
      case BC_PERIODIC: return g - n;
      case BC_EXTRAP: return n - 1;
      default: *flip = 1; return 2 * n - 1 - g;
    }
  }
  return g;
}

/* Load the conservative state of cell idx, where idx[d] may lie in a ghost
 * layer of axis d. */
static void load_cons(const orc_problem* P, const double* q, int d, const int idx[3], double* U) {
  int neq = orc_num_eqs(P);
  int flip = 0;
  int id[3] = {idx[0], idx[1], idx[2]};
  id[d] = ghost_map(P, d, idx[d], &flip);
  int64_t nc = ncell(P);
  int64_t c = ((int64_t)id[2] * P->n[1] + id[1]) * P->n[0] + id[0];
  for (int v = 0; v < neq; ++v) U[v] = q[v * nc + c];
  if (flip) U[row_mom(P, d)] = -U[row_mom(P, d)];
}

/* Width of cell position g along axis d (g may lie in a ghost layer).  A   */
/* ghost cell takes the width of the interior cell whose state it holds     */
/* (the same index map as the state: wrap, nearest cell, or mirror image);  */
/* reading: the paper states no ghost widths for non-uniform grids.         */
static double cell_width(const orc_problem* P, int d, int g) {
  if (!P->faces[d]) return P->dx[d];
  int flip = 0;
  int i = ghost_map(P, d, g, &flip);
  return P->faces[d][i + 1] - P->faces[d][i];
}

/* ------------------------------------------------------------------------ */
/* WENO5-JS (Sec. 3.2.1; Jiang-Shu weights as in Shu's 1997 report).       */
/* Left-biased value at the face right of the centre cell from the five     */
/* cell values f[0..4] = f_{i-2..i+2}: three third-order candidates, the    */
/* smoothness indicators beta_k, weights a_k = d_k/(eps + beta_k)^2 with    */
/* linear weights d = (0.1, 0.6, 0.3), and their normalized combination.    */
/* The beta_k are written with commuted sums so that the reversed stencil   */
/* yields the same three numbers (beta_0 <-> beta_2).                       */
/* ------------------------------------------------------------------------ */
static double sq(double x) { return x * x; }

double orc_weno5_js_left(const double* f, double eps) {
  double a = f[0], b = f[1], c = f[2], d = f[3], e = f[4];
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double b0 = 13.0 / 12.0 * sq((a + c) - 2.0 * b) + 0.25 * sq((a + 3.0 * c) - 4.0 * b);
  double b1 = 13.0 / 12.0 * sq((b + d) - 2.0 * c) + 0.25 * sq(b - d);
  double b2 = 13.0 / 12.0 * sq((c + e) - 2.0 * d) + 0.25 * sq((3.0 * c + e) - 4.0 * d);
  double a0 = 0.1 / sq(eps + b0);
  double a1 = 0.6 / sq(eps + b1);
  double a2 = 0.3 / sq(eps + b2);
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* Right-biased value at the face left of the centre: the mirror image. */
double orc_weno5_js_right(const double* f, double eps) {
  double r[5] = {f[4], f[3], f[2], f[1], f[0]};
  return orc_weno5_js_left(r, eps);
}

/* ------------------------------------------------------------------------ */
/* WENO5-Z (Sec. 4.2.2, the Borges et al. weights as the paper prints them  */
/* for order 2k-1 = 5): the same candidates and smoothness indicators as    */
/* above, the global indicator tau = |beta_0 - beta_2|, and weights          */
/* a_k = d_k (1 + (tau/(beta_k + eps))^q) with q = 1, normalized.            */
/* ------------------------------------------------------------------------ */
double orc_weno5_z_left(const double* f, double eps) {
  double a = f[0], b = f[1], c = f[2], d = f[3], e = f[4];
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double b0 = 13.0 / 12.0 * sq((a + c) - 2.0 * b) + 0.25 * sq((a + 3.0 * c) - 4.0 * b);
  double b1 = 13.0 / 12.0 * sq((b + d) - 2.0 * c) + 0.25 * sq(b - d);
  double b2 = 13.0 / 12.0 * sq((c + e) - 2.0 * d) + 0.25 * sq((3.0 * c + e) - 4.0 * d);
  double tau = fabs(b0 - b2);
  double a0 = 0.1 * (1.0 + tau / (b0 + eps));
  double a1 = 0.6 * (1.0 + tau / (b1 + eps));
  double a2 = 0.3 * (1.0 + tau / (b2 + eps));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

double orc_weno5_z_right(const double* f, double eps) {
  double r[5] = {f[4], f[3], f[2], f[1], f[0]};
  return orc_weno5_z_left(r, eps);
}

/* ------------------------------------------------------------------------ */
/* WENO5-M.  Sec. 3.2.1 keeps fifth order through the mapped weights of      */
/* Henrick, Aslam and Powers (2005), which it cites without printing them.   */
/* Their definition: the JS weights w_k = a_k / sum a are mapped by           */
/*   g_k(w) = w (d_k + d_k^2 - 3 d_k w + w^2) / (d_k^2 + w (1 - 2 d_k)),     */
/* which fixes 0, d_k and 1 and is flat to second order at d_k, and the       */
/* mapped values are normalized again.  Same candidates, indicators and eps. */
/* ------------------------------------------------------------------------ */
double orc_weno_m_map(double w, double d) {
  return w * (d + d * d - 3.0 * d * w + w * w) / (d * d + w * (1.0 - 2.0 * d));
}

double orc_weno5_m_left(const double* f, double eps) {
  double a = f[0], b = f[1], c = f[2], d = f[3], e = f[4];
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double b0 = 13.0 / 12.0 * sq((a + c) - 2.0 * b) + 0.25 * sq((a + 3.0 * c) - 4.0 * b);
  double b1 = 13.0 / 12.0 * sq((b + d) - 2.0 * c) + 0.25 * sq(b - d);
  double b2 = 13.0 / 12.0 * sq((c + e) - 2.0 * d) + 0.25 * sq((3.0 * c + e) - 4.0 * d);
  double a0 = 0.1 / sq(eps + b0);
  double a1 = 0.6 / sq(eps + b1);
  double a2 = 0.3 / sq(eps + b2);
  double as = a0 + a1 + a2;
  double m0 = orc_weno_m_map(a0 / as, 0.1);
  double m1 = orc_weno_m_map(a1 / as, 0.6);
  double m2 = orc_weno_m_map(a2 / as, 0.3);
  return (m0 * q0 + m1 * q1 + m2 * q2) / (m0 + m1 + m2);
}

double orc_weno5_m_right(const double* f, double eps) {
  double r[5] = {f[4], f[3], f[2], f[1], f[0]};
  return orc_weno5_m_left(r, eps);
}

/* ------------------------------------------------------------------------ */
/* TENO5 (Sec. 4.2.2): the same three candidates and indicators; a stencil   */
/* takes part (delta_r = 1) when its share chi_r = gamma_r / sum gamma of    */
/* gamma_r = d_r (1 + tau/(beta_r + eps))^6 reaches the cut-off C_T, and the  */
/* kept stencils combine with their linear weights, d_r delta_r / sum d delta.*/
/* ------------------------------------------------------------------------ */
static double pow6(double x) {
  double x2 = x * x;
  return x2 * x2 * x2;
}

double orc_teno5_left(const double* f, double eps, double ct) {
  double a = f[0], b = f[1], c = f[2], d = f[3], e = f[4];
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double b0 = 13.0 / 12.0 * sq((a + c) - 2.0 * b) + 0.25 * sq((a + 3.0 * c) - 4.0 * b);
  double b1 = 13.0 / 12.0 * sq((b + d) - 2.0 * c) + 0.25 * sq(b - d);
  double b2 = 13.0 / 12.0 * sq((c + e) - 2.0 * d) + 0.25 * sq((3.0 * c + e) - 4.0 * d);
  double tau = fabs(b0 - b2);
  double g0 = 0.1 * pow6(1.0 + tau / (b0 + eps));
  double g1 = 0.6 * pow6(1.0 + tau / (b1 + eps));
  double g2 = 0.3 * pow6(1.0 + tau / (b2 + eps));
  double gs = g0 + g1 + g2;
  double w0 = (g0 / gs >= ct) ? 0.1 : 0.0;
  double w1 = (g1 / gs >= ct) ? 0.6 : 0.0;
  double w2 = (g2 / gs >= ct) ? 0.3 : 0.0;
  return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

double orc_teno5_right(const double* f, double eps, double ct) {
  double r[5] = {f[4], f[3], f[2], f[1], f[0]};
  return orc_teno5_left(r, eps, ct);
}

/* ------------------------------------------------------------------------ */
/* Fifth-order reconstruction on a non-uniform grid (Sec. 4.2.2), from the   */
/* Lagrange form the paper prints.  For K cells with faces x_0 < .. < x_K,  */
/* widths h_j and averages f_j, the primitive P(x_m) = sum_{j<m} h_j f_j is  */
/* interpolated at the K + 1 faces by the Lagrange basis L_m, and the        */
/* reconstruction polynomial is its derivative,                              */
/*   p(x) = sum_m P(x_m) L_m'(x) = sum_j h_j sum_{m>j} L_m'(x) f_j,          */
/* which is the paper's c_j(x).  Derivatives of L_m are formed from the     */
/* product rule: the s-th derivative of prod_{i}(x - z_i) is s! times the    */
/* sum over the ways of dropping s factors of the product of the rest.      */
/* ------------------------------------------------------------------------ */
static double prod_deriv(const double* z, int nz, int s, double x) {
  double total = 0.0;
  for (int mask = 0; mask < (1 << nz); ++mask) {
    if (__builtin_popcount(mask) != s) continue;
    double pr = 1.0;
    for (int i = 0; i < nz; ++i)
      if (!((mask >> i) & 1)) pr = pr * (x - z[i]);
    total = total + pr;
  }
  double fact = 1.0;
  for (int i = 2; i <= s; ++i) fact = fact * i;
  return total * fact;
}

/* s-th derivative of the Lagrange basis polynomial L_m on nodes x[0..K]. */
static double lagrange_deriv(const double* x, int K, int m, int s, double at) {
  double z[8], den = 1.0;
  int nz = 0;
  for (int l = 0; l <= K; ++l) {
    if (l == m) continue;
    z[nz++] = x[l];
    den = den * (x[m] - x[l]);
  }
  return prod_deriv(z, nz, s, at) / den;
}

/* Coefficient of f_j in the l-th derivative of the reconstruction polynomial
 * of the K cells with faces x[0..K] (l = 0: the value). */
static double recon_coef(const double* x, int K, int j, int l, double at) {
  double h = x[j + 1] - x[j], c = 0.0;
  for (int m = j + 1; m <= K; ++m) c = c + lagrange_deriv(x, K, m, l + 1, at);
  return h * c;
}

/* The candidates, smoothness indicators and ideal weights of the fifth-order
 * reconstruction at the centre cell of five cells with widths h[0..4] and
 * averages f[0..4] (centre: cell 2).  Stencil r covers cells r..r+2.
 *   qR[r], qL[r]: candidate r at the right and at the left face of the centre;
 *   beta[r] = sum_{l=1,2} h_c^(2l-1) int_cell (p_r^(l))^2 dx, the integral by
 *     two-point Gauss-Legendre quadrature (exact: the integrands are
 *     polynomials of degree at most two);
 *   dR[r], dL[r]: ideal weights at the two faces.  Reading (the paper names
 *     them without a formula for non-uniform grids): the weights for which
 *     sum_r d_r p_r equals the five-cell reconstruction at that face for all
 *     data; f_0 enters only stencil 0 and f_4 only stencil 2, so d_0 and d_2
 *     are those coefficient ratios and d_1 = 1 - d_0 - d_2.  A uniform grid
 *     gives (0.1, 0.6, 0.3) at the right face and (0.3, 0.6, 0.1) at the left.
 * f may be NULL (coefficients only: qR, qL and beta are then not formed). */
void orc_nu_stencil(const double* f, const double* h, double* qR, double* qL, double* beta, double* dR,
                    double* dL) {
  double x[6];
  x[0] = 0.0;
  for (int j = 0; j < 5; ++j) x[j + 1] = x[j] + h[j];
  double xl = x[2], xr = x[3], hc = h[2];
  double g = 0.5 / sqrt(3.0);
  double gp[2] = {0.5 * (xl + xr) - g * hc, 0.5 * (xl + xr) + g * hc};
  for (int r = 0; r < 3; ++r) {
    const double* xs = &x[r];
    if (f) {
      double vr = 0.0, vl = 0.0;
      for (int j = 0; j < 3; ++j) {
        vr = vr + recon_coef(xs, 3, j, 0, xr) * f[r + j];
        vl = vl + recon_coef(xs, 3, j, 0, xl) * f[r + j];
      }
      qR[r] = vr;
      qL[r] = vl;
      double b = 0.0;
      for (int l = 1; l <= 2; ++l) {
        double integral = 0.0;
        for (int k = 0; k < 2; ++k) {
          double dv = 0.0;
          for (int j = 0; j < 3; ++j) dv = dv + recon_coef(xs, 3, j, l, gp[k]) * f[r + j];
          integral = integral + 0.5 * hc * dv * dv;
        }
        b = b + pow(hc, 2 * l - 1) * integral;
      }
      beta[r] = b;
    }
  }
  double at[2] = {xr, xl};
  double* dout[2] = {dR, dL};
  for (int side = 0; side < 2; ++side) {
    double c5_first = recon_coef(x, 5, 0, 0, at[side]);
    double c5_last = recon_coef(x, 5, 4, 0, at[side]);
    double c3_first = recon_coef(&x[0], 3, 0, 0, at[side]);
    double c3_last = recon_coef(&x[2], 3, 2, 0, at[side]);
    double d0 = c5_first / c3_first, d2 = c5_last / c3_last;
    dout[side][0] = d0;
    dout[side][1] = 1.0 - d0 - d2;
    dout[side][2] = d2;
  }
}

/* WENO5-JS on a non-uniform grid: Jiang-Shu weights d_r/(eps + beta_r)^2 of
 * the quantities above, normalized, at the right face (fR, the left state of
 * the face right of the centre) and at the left face (fL). */
void orc_weno5_nu(const double* f, const double* h, double eps, double* fR, double* fL) {
  double qR[3], qL[3], beta[3], dR[3], dL[3];
  orc_nu_stencil(f, h, qR, qL, beta, dR, dL);
  double numR = 0.0, denR = 0.0, numL = 0.0, denL = 0.0;
  for (int r = 0; r < 3; ++r) {
    double aR = dR[r] / sq(eps + beta[r]);
    double aL = dL[r] / sq(eps + beta[r]);
    numR = numR + aR * qR[r];
    denR = denR + aR;
    numL = numL + aL * qL[r];
    denL = denL + aL;
  }
  *fR = numR / denR;
  *fL = numL / denL;
}

/* ------------------------------------------------------------------------ */
/* HLLC face solver (Sec. 3.2.2; star states from Toro's book, the paper's  */
/* reference for the solver).  Returns the flux of every row and the face   */
/* velocity u_f that the non-conservative alpha term uses (Sec. 3.2.1: the  */
/* Riemann problem yields F and u at the face).                             */
/* Readings:                                                                */
/*   wave speeds: S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L,     */
/*     u_R + c_R) (the form printed for HLLD in Sec. 4.2.5); ties take the  */
/*     first argument;                                                      */
/*   contact speed S* from continuity of normal velocity and pressure;      */
/*   regions: S_L >= 0 -> left; S* >= 0 -> left star; S_R > 0 -> right star;*/
/*     else right (the flux is continuous at each boundary);                */
/*   volume fractions ride the contact: flux alpha_K u_f with K the side    */
/*     the face takes, u_f = u_L, S*, S*, u_R in the four regions.          */
/* Returns 0, or 1 if a face state has c^2 <= 0 or a flux is not finite.    */
/* ------------------------------------------------------------------------ */
typedef struct {
  double rho, un, p, E, c, Gam, Pi;
  double U[NEQ_MAX], F[NEQ_MAX];
} face_state;

static int face_side(const orc_problem* P, int d, const double* W, face_state* s) {
  int nf = P->num_fluids, D = P->ndim;
  double rho = 0.0;
  for (int i = 0; i < nf; ++i) rho = rho + W[i];
  double usq = 0.0;
  for (int e = 0; e < D; ++e) usq = usq + W[row_mom(P, e)] * W[row_mom(P, e)];
  double Gam, Pi;
  mixture(P, nf == 2 ? &W[row_alpha(P, 0)] : NULL, &Gam, &Pi);
  double p = W[row_E(P)];
  double un = W[row_mom(P, d)];
  double E = Gam * p + Pi + 0.5 * rho * usq;
  double c2 = sound_speed_sq(rho, p, Gam, Pi);
  s->rho = rho;
  s->un = un;
  s->p = p;
  s->E = E;
  s->Gam = Gam;
  s->Pi = Pi;
  s->c = sqrt(c2);
  for (int i = 0; i < nf; ++i) {
    s->U[i] = W[i];
    s->F[i] = W[i] * un;
  }
  for (int e = 0; e < D; ++e) {
    double m = rho * W[row_mom(P, e)];
    s->U[row_mom(P, e)] = m;
    s->F[row_mom(P, e)] = m * un + (e == d ? p : 0.0);
  }
  s->U[row_E(P)] = E;
  s->F[row_E(P)] = (E + p) * un;
  return !(c2 > 0.0);
}

/* Star state U*_K of side K (Toro): chi = (S_K - u_K)/(S_K - S*). */
static void star_state(const orc_problem* P, int d, const double* W, const face_state* s,
                       double SK, double Sstar, double* Us) {
  int nf = P->num_fluids, D = P->ndim;
  double chi = (SK - s->un) / (SK - Sstar);
  for (int i = 0; i < nf; ++i) Us[i] = chi * W[i];
  for (int e = 0; e < D; ++e)
    Us[row_mom(P, e)] = (e == d) ? chi * s->rho * Sstar : chi * s->rho * W[row_mom(P, e)];
  Us[row_E(P)] = chi * (s->E + (Sstar - s->un) * (s->rho * Sstar + s->p / (SK - s->un)));
}

int orc_hllc(const orc_problem* P, int d, const double* WL, const double* WR, double* F,
             double* uf) {
  int nf = P->num_fluids, neq = orc_num_eqs(P);
  int ncons = row_E(P) + 1;
  face_state L, R;
  int bad = face_side(P, d, WL, &L);
  bad |= face_side(P, d, WR, &R);
  double sl_a = L.un - L.c, sl_b = R.un - R.c;
  double sr_a = L.un + L.c, sr_b = R.un + R.c;
  double SL = (sl_a <= sl_b) ? sl_a : sl_b;
  double SR = (sr_a >= sr_b) ? sr_a : sr_b;
  double Sstar = (R.p - L.p + L.rho * L.un * (SL - L.un) - R.rho * R.un * (SR - R.un)) /
                 (L.rho * (SL - L.un) - R.rho * (SR - R.un));
  double Us[NEQ_MAX];
  const double* alpha_side;
  /* Anti-dissipation pressure correction of Chen et al. (Sec. 4.2.4), added
   * to both star-region fluxes:
   *   p_d = rho_L rho_R (S_L - u_L)(S_R - u_R)(u_R - u_L)
   *         / (rho_R (S_R - u_R) - rho_L (S_L - u_L)),
   *   APC = (z - 1) p_d on the face-normal momentum, (z - 1) p_d S* on the
   *   energy, with z = min(max(|u_L|/c_L, |u_R|/c_R), 1) (the Mach number of
   *   the low-Mach section; sound speeds of the reconstructed states). */
  double apc_mom = 0.0, apc_E = 0.0;
  if (P->low_mach == 2) {
    double mL = fabs(L.un) / L.c, mR = fabs(R.un) / R.c;
    double z = (mL >= mR) ? mL : mR;
    if (z > 1.0) z = 1.0;
    double pd = L.rho * R.rho * (SL - L.un) * (SR - R.un) * (R.un - L.un) /
                (R.rho * (SR - R.un) - L.rho * (SL - L.un));
    apc_mom = (z - 1.0) * pd;
    apc_E = (z - 1.0) * pd * Sstar;
  }
  if (SL >= 0.0) {
    for (int v = 0; v < ncons; ++v) F[v] = L.F[v];
    *uf = L.un;
    alpha_side = WL;
  } else if (Sstar >= 0.0) {
    star_state(P, d, WL, &L, SL, Sstar, Us);
    for (int v = 0; v < ncons; ++v) F[v] = L.F[v] + SL * (Us[v] - L.U[v]);
    if (P->low_mach == 2) {
      F[row_mom(P, d)] = F[row_mom(P, d)] + apc_mom;
      F[row_E(P)] = F[row_E(P)] + apc_E;
    }
    *uf = Sstar;
    alpha_side = WL;
  } else if (SR > 0.0) {
    star_state(P, d, WR, &R, SR, Sstar, Us);
    for (int v = 0; v < ncons; ++v) F[v] = R.F[v] + SR * (Us[v] - R.U[v]);
    if (P->low_mach == 2) {
      F[row_mom(P, d)] = F[row_mom(P, d)] + apc_mom;
      F[row_E(P)] = F[row_E(P)] + apc_E;
    }
    *uf = Sstar;
    alpha_side = WR;
  } else {
    for (int v = 0; v < ncons; ++v) F[v] = R.F[v];
    *uf = R.un;
    alpha_side = WR;
  }
  if (nf == 2)
    for (int i = 0; i < 2; ++i) F[row_alpha(P, i)] = alpha_side[row_alpha(P, i)] * (*uf);
  for (int v = 0; v < neq; ++v)
    if (!isfinite(F[v])) bad = 1;
  if (!isfinite(*uf)) bad = 1;
  return bad;
}

/* ------------------------------------------------------------------------ */
/* HLL face solver (Sec. 3.2.2, from Toro's book): two waves S_L, S_R, the  */
/* same estimates as HLLC, and one averaged state between them (no contact):*/
/*   F = F_L if S_L >= 0, F_R if S_R <= 0, else                              */
/*   F = (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).             */
/* Readings (the paper prints no formula): the volume fractions take the    */
/* same formula on their advective flux alpha u_n, and the face velocity of */
/* the alpha source is the matching average u_f = (S_R u_L - S_L u_R) /     */
/* (S_R - S_L) (u_L or u_R in the one-sided cases), so that a uniform alpha */
/* stays uniform.                                                           */
/* ------------------------------------------------------------------------ */
int orc_hll(const orc_problem* P, int d, const double* WL, const double* WR, double* F, double* uf) {
  int nf = P->num_fluids, neq = orc_num_eqs(P);
  int ncons = row_E(P) + 1;
  face_state L, R;
  int bad = face_side(P, d, WL, &L);
  bad |= face_side(P, d, WR, &R);
  double sl_a = L.un - L.c, sl_b = R.un - R.c;
  double sr_a = L.un + L.c, sr_b = R.un + R.c;
  double SL = (sl_a <= sl_b) ? sl_a : sl_b;
  double SR = (sr_a >= sr_b) ? sr_a : sr_b;
  if (SL >= 0.0) {
    for (int v = 0; v < ncons; ++v) F[v] = L.F[v];
    *uf = L.un;
    if (nf == 2)
      for (int i = 0; i < 2; ++i) F[row_alpha(P, i)] = WL[row_alpha(P, i)] * L.un;
  } else if (SR <= 0.0) {
    for (int v = 0; v < ncons; ++v) F[v] = R.F[v];
    *uf = R.un;
    if (nf == 2)
      for (int i = 0; i < 2; ++i) F[row_alpha(P, i)] = WR[row_alpha(P, i)] * R.un;
  } else {
    double den = SR - SL;
    for (int v = 0; v < ncons; ++v) F[v] = (SR * L.F[v] - SL * R.F[v] + SL * SR * (R.U[v] - L.U[v])) / den;
    *uf = (SR * L.un - SL * R.un) / den;
    if (nf == 2)
      for (int i = 0; i < 2; ++i) {
        double aL = WL[row_alpha(P, i)], aR = WR[row_alpha(P, i)];
        F[row_alpha(P, i)] = (SR * aL * L.un - SL * aR * R.un + SL * SR * (aR - aL)) / den;
      }
  }
  for (int v = 0; v < neq; ++v)
    if (!isfinite(F[v])) bad = 1;
  if (!isfinite(*uf)) bad = 1;
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Low-Mach correction of Thornber et al., as the paper prints it (Sec. 4.2,*/
/* low-Mach treatment): with z = min(max(|u_L|/c_L, |u_R|/c_R), 1) the face-*/
/* normal velocities of the two reconstructed states become                 */
/*   u_L* = (u_L + u_R)/2 + z (u_L - u_R)/2,  u_R* = (u_L + u_R)/2 + z (u_R - u_L)/2,*/
/* and replace u_L, u_R in the face solver (wave speeds and fluxes).        */
/* Reading: c_L, c_R are the sound speeds of the uncorrected states.        */
/* ------------------------------------------------------------------------ */
void orc_thornber(const orc_problem* P, int d, double* WL, double* WR) {
  face_state L, R;
  face_side(P, d, WL, &L);
  face_side(P, d, WR, &R);
  double mL = fabs(L.un) / L.c, mR = fabs(R.un) / R.c;
  double z = (mL >= mR) ? mL : mR;
  if (z > 1.0) z = 1.0;
  double uL = WL[row_mom(P, d)], uR = WR[row_mom(P, d)];
  WL[row_mom(P, d)] = 0.5 * (uL + uR) + z * (0.5 * (uL - uR));
  WR[row_mom(P, d)] = 0.5 * (uL + uR) + z * (0.5 * (uR - uL));
}

/* ------------------------------------------------------------------------ */
/* Face flux along axis d at the face on the low side of cell idx (face     */
/* m - 1/2 with m = idx[d]): cells m-3..m+2 are loaded (ghost layers mapped),*/
/* converted to primitive variables, reconstructed component-wise (left     */
/* state from centre m-1, right state from centre m), and handed to HLLC.   */
/* ------------------------------------------------------------------------ */
static int face_flux(const orc_problem* P, const double* q, int d, const int idx[3], double* F,
                     double* uf) {
  int neq = orc_num_eqs(P);
  double Wc[6][NEQ_MAX];
  for (int s = 0; s < 6; ++s) {
    int id[3] = {idx[0], idx[1], idx[2]};
    id[d] = idx[d] - 3 + s;
    double U[NEQ_MAX];
    load_cons(P, q, d, id, U);
    cell_cons_to_prim(P, U, Wc[s]);
  }
  double WL[NEQ_MAX], WR[NEQ_MAX];
  double hl[5], hr[5];
  if (P->faces[d])
    for (int s = 0; s < 5; ++s) {
      hl[s] = cell_width(P, d, idx[d] - 3 + s);
      hr[s] = cell_width(P, d, idx[d] - 2 + s);
    }
  for (int v = 0; v < neq; ++v) {
    double fl[5], fr[5];
    for (int s = 0; s < 5; ++s) {
      fl[s] = Wc[s][v];      /* centre m-1: cells m-3..m+1 */
      fr[s] = Wc[s + 1][v];  /* centre m:   cells m-2..m+2 */
    }
    if (P->faces[d]) {
      double unused;
      orc_weno5_nu(fl, hl, P->weno_eps, &WL[v], &unused);
      orc_weno5_nu(fr, hr, P->weno_eps, &unused, &WR[v]);
    } else if (P->weno_variant == 1) {
      WL[v] = orc_weno5_z_left(fl, P->weno_eps);
      WR[v] = orc_weno5_z_right(fr, P->weno_eps);
    } else if (P->weno_variant == 2) {
      WL[v] = orc_teno5_left(fl, P->weno_eps, ORC_TENO_CT);
      WR[v] = orc_teno5_right(fr, P->weno_eps, ORC_TENO_CT);
    } else if (P->weno_variant == 3) {
      WL[v] = orc_weno5_m_left(fl, P->weno_eps);
      WR[v] = orc_weno5_m_right(fr, P->weno_eps);
    } else {
      WL[v] = orc_weno5_js_left(fl, P->weno_eps);
      WR[v] = orc_weno5_js_right(fr, P->weno_eps);
    }
  }
  if (P->low_mach == 1) orc_thornber(P, d, WL, WR);
  return P->riemann == 1 ? orc_hll(P, d, WL, WR, F, uf) : orc_hllc(P, d, WL, WR, F, uf);
}

/* ------------------------------------------------------------------------ */
/* Kapila's K (Sec. 2.1.1): the alpha_1 equation of the five-equation model  */
/* carries K div u with                                                     */
/*   K = (rho_2 c_2^2 - rho_1 c_1^2) / (rho_1 c_1^2/alpha_1 + rho_2 c_2^2/alpha_2),*/
/* phasic densities rho_i = (alpha_i rho_i)/alpha_i and phasic sound speeds  */
/* c_i = sqrt(gamma_i (p + pi_inf,i)/rho_i).  Reading: the printed numerator */
/* has a plus sign, which would not vanish for two identical fluids; the     */
/* thermodynamically consistent term (each phase compressed along its own    */
/* isentrope) has the difference, as written here.  The alpha_2 equation     */
/* takes -K, so that alpha_1 + alpha_2 is unchanged.  W: primitive state of  */
/* the cell (cell averages).                                                */
/* ------------------------------------------------------------------------ */
double orc_kapila_K(const orc_problem* P, const double* W) {
  double p = W[row_E(P)];
  double rc2[2];
  for (int i = 0; i < 2; ++i) {
    double alpha = W[row_alpha(P, i)];
    double rho_i = W[i] / alpha;
    double c2_i = P->gamma[i] * (p + P->pi_inf[i]) / rho_i;
    rc2[i] = rho_i * c2_i;
  }
  double a1 = W[row_alpha(P, 0)], a2 = W[row_alpha(P, 1)];
  return (rc2[1] - rc2[0]) / (rc2[0] / a1 + rc2[1] / a2);
}

/* Contribution of axis d to the RHS of one cell (eq. eqn:rhs with s = 0 and
 * h = -alpha for the Allaire model, K = 0; h = -(alpha_i + K_i) with K_1 = K,
 * K_2 = -K for the Kapila model):
 *   D_v = (F_{m-1/2} - F_{m+1/2}) / dx_d for every row,
 *   plus alpha_cell (u_{m+1/2} - u_{m-1/2}) / dx_d on the alpha rows, where
 *   alpha_cell is the cell-average volume fraction. */
static void axis_contribution(const orc_problem* P, int d, int i_d, const double* Flo, double ulo,
                              const double* Fhi, double uhi, const double* Ucell,
                              double* Dv) {
  int nf = P->num_fluids, neq = orc_num_eqs(P);
  double inv_dx = 1.0 / cell_width(P, d, i_d);
  for (int v = 0; v < neq; ++v) Dv[v] = inv_dx * (Flo[v] - Fhi[v]);
  if (nf == 2) {
    double K[2] = {0.0, 0.0};
    if (P->model == 1) {
      double Wc[NEQ_MAX];
      cell_cons_to_prim(P, Ucell, Wc);
      K[0] = orc_kapila_K(P, Wc);
      K[1] = -K[0];
    }
    for (int i = 0; i < 2; ++i) {
      int a = row_alpha(P, i);
      if (P->model == 1)
        Dv[a] = Dv[a] + (Ucell[a] + K[i]) * (inv_dx * (uhi - ulo));
      else
        Dv[a] = Dv[a] + Ucell[a] * (inv_dx * (uhi - ulo));
    }
  }
}

/* Full RHS: rhs = sum over axes d = 0..D-1 (in that order) of D_d. */
int orc_rhs(const orc_problem* P, const double* q, double* rhs) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P);
  int bad = 0;
  memset(rhs, 0, sizeof(double) * (size_t)neq * (size_t)nc);
  for (int d = 0; d < P->ndim; ++d) {
    int nd = P->n[d];
    /* lines along d: enumerate cells with idx[d] == 0 */
    int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    int64_t nlines = (int64_t)P->n[e1] * P->n[e2];
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t line = 0; line < nlines; ++line) {
      int idx[3];
      idx[d] = 0;
      idx[e1] = (int)(line % P->n[e1]);
      idx[e2] = (int)(line / P->n[e1]);
      double* Fl = (double*)malloc(sizeof(double) * (size_t)(nd + 1) * NEQ_MAX);
      double* ul = (double*)malloc(sizeof(double) * (size_t)(nd + 1));
      for (int m = 0; m <= nd; ++m) {
        int id[3] = {idx[0], idx[1], idx[2]};
        id[d] = m;
        bad |= face_flux(P, q, d, id, &Fl[(size_t)m * NEQ_MAX], &ul[m]);
      }
      for (int m = 0; m < nd; ++m) {
        int id[3] = {idx[0], idx[1], idx[2]};
        id[d] = m;
        int64_t c = ((int64_t)id[2] * P->n[1] + id[1]) * P->n[0] + id[0];
        double Uc[NEQ_MAX], Dv[NEQ_MAX];
        for (int v = 0; v < neq; ++v) Uc[v] = q[v * nc + c];
        axis_contribution(P, d, m, &Fl[(size_t)m * NEQ_MAX], ul[m], &Fl[(size_t)(m + 1) * NEQ_MAX],
                          ul[m + 1], Uc, Dv);
        for (int v = 0; v < neq; ++v) rhs[v * nc + c] = rhs[v * nc + c] + Dv[v];
      }
      free(Fl);
      free(ul);
    }
  }
  return bad ? ORC_ERR_NONFINITE : ORC_OK;
}

/* RHS at selected cells only (same arithmetic as orc_rhs, face by face).
 * cells: linear indices k*ny*nx + j*nx + i; out: [ncells][neq]. */
int orc_rhs_cells(const orc_problem* P, const double* q, int64_t ncells, const int64_t* cells,
                  double* out) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int64_t s = 0; s < ncells; ++s) {
    int64_t c = cells[s];
    int idx[3] = {(int)(c % P->n[0]), (int)((c / P->n[0]) % P->n[1]),
                  (int)(c / ((int64_t)P->n[0] * P->n[1]))};
    double acc[NEQ_MAX], Uc[NEQ_MAX];
    for (int v = 0; v < neq; ++v) {
      acc[v] = 0.0;
      Uc[v] = q[v * nc + c];
    }
    for (int d = 0; d < P->ndim; ++d) {
      double Flo[NEQ_MAX], Fhi[NEQ_MAX], ulo, uhi, Dv[NEQ_MAX];
      int id[3] = {idx[0], idx[1], idx[2]};
      bad |= face_flux(P, q, d, id, Flo, &ulo);
      id[d] = idx[d] + 1;
      bad |= face_flux(P, q, d, id, Fhi, &uhi);
      axis_contribution(P, d, idx[d], Flo, ulo, Fhi, uhi, Uc, Dv);
      for (int v = 0; v < neq; ++v) acc[v] = acc[v] + Dv[v];
    }
    for (int v = 0; v < neq; ++v) out[s * neq + v] = acc[v];
  }
  return bad ? ORC_ERR_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Signal speed for the time step (the paper gives no rule; reading: the    */
/* unsplit sum form s = max over cells of sum_d (|u_d| + c)/dx_d, with      */
/* dt = CFL/s).                                                             */
/* ------------------------------------------------------------------------ */
int orc_max_signal(const orc_problem* P, const double* q, double* smax_out) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P), nf = P->num_fluids;
  int64_t nc = ncell(P);
  double smax = 0.0;
  int bad = 0;
#pragma omp parallel for reduction(max : smax) reduction(| : bad)
  for (int64_t c = 0; c < nc; ++c) {
    double U[NEQ_MAX], W[NEQ_MAX];
    for (int v = 0; v < neq; ++v) U[v] = q[v * nc + c];
    cell_cons_to_prim(P, U, W);
    double rho = 0.0;
    for (int i = 0; i < nf; ++i) rho = rho + U[i];
    double Gam, Pi;
    mixture(P, nf == 2 ? &U[row_alpha(P, 0)] : NULL, &Gam, &Pi);
    double c2 = sound_speed_sq(rho, W[row_E(P)], Gam, Pi);
    if (!(c2 > 0.0) || !isfinite(c2)) bad = 1;
    double cs = sqrt(c2);
    int idx[3] = {(int)(c % P->n[0]), (int)((c / P->n[0]) % P->n[1]),
                  (int)(c / ((int64_t)P->n[0] * P->n[1]))};
    double s = 0.0;
    for (int d = 0; d < P->ndim; ++d) s = s + (fabs(W[row_mom(P, d)]) + cs) * (1.0 / cell_width(P, d, idx[d]));
    if (!isfinite(s)) bad = 1;
    if (s > smax) smax = s;
  }
  *smax_out = smax;
  return bad ? ORC_ERR_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SSP-RK3 step, Shu-Osher form (Sec. 3.4; Gottlieb-Shu 1998):             */
/*   q1 = qn + dt L(qn)                                                     */
/*   q2 = 3/4 qn + 1/4 (q1 + dt L(q1))                                      */
/*   q^{n+1} = 1/3 qn + 2/3 (q2 + dt L(q2))                                 */
/* dt: cfl > 0 -> CFL/s (clipped to t_remaining when that is > 0);          */
/*     otherwise dt_fixed.  Exactly one of cfl, dt_fixed must be positive.  */
/* ------------------------------------------------------------------------ */
int orc_step(const orc_problem* P, double* q, double cfl, double dt_fixed, double t_remaining,
             double* dt_out) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  if ((cfl > 0) == (dt_fixed > 0)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P), ne = (int64_t)neq * nc;
  int bad = 0;
  double dt = dt_fixed;
  if (cfl > 0) {
    double s;
    bad |= orc_max_signal(P, q, &s) != ORC_OK;
    dt = cfl / s;
    if (t_remaining > 0 && dt > t_remaining) dt = t_remaining;
  }
  double* L = (double*)malloc(sizeof(double) * (size_t)ne);
  double* q1 = (double*)malloc(sizeof(double) * (size_t)ne);
  double* q2 = (double*)malloc(sizeof(double) * (size_t)ne);
  bad |= orc_rhs(P, q, L) != ORC_OK;
#pragma omp parallel for
  for (int64_t e = 0; e < ne; ++e) q1[e] = q[e] + dt * L[e];
  bad |= orc_rhs(P, q1, L) != ORC_OK;
#pragma omp parallel for
  for (int64_t e = 0; e < ne; ++e) q2[e] = 0.75 * q[e] + 0.25 * (q1[e] + dt * L[e]);
  bad |= orc_rhs(P, q2, L) != ORC_OK;
#pragma omp parallel for
  for (int64_t e = 0; e < ne; ++e) q[e] = (1.0 / 3.0) * q[e] + (2.0 / 3.0) * (q2[e] + dt * L[e]);
  free(L);
  free(q1);
  free(q2);
  if (dt_out) *dt_out = dt;
  return bad ? ORC_ERR_NONFINITE : ORC_OK;
}

/* Run `nsteps` steps; dts (optional, length nsteps) receives each dt. */
int orc_run(const orc_problem* P, double* q, int nsteps, double cfl, double dt_fixed,
            double* dts) {
  int rc = ORC_OK;
  for (int s = 0; s < nsteps; ++s) {
    double dt;
    int r = orc_step(P, q, cfl, dt_fixed, 0.0, &dt);
    if (r == ORC_ERR_ARG) return r;
    if (r != ORC_OK) rc = r;
    if (dts) dts[s] = dt;
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Field conversions and diagnostics                                        */
/* ------------------------------------------------------------------------ */
int orc_prim_to_cons(const orc_problem* P, const double* w, double* q) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c) {
    double W[NEQ_MAX], U[NEQ_MAX];
    for (int v = 0; v < neq; ++v) W[v] = w[v * nc + c];
    cell_prim_to_cons(P, W, U);
    for (int v = 0; v < neq; ++v) q[v * nc + c] = U[v];
  }
  return ORC_OK;
}

int orc_cons_to_prim(const orc_problem* P, const double* q, double* w) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c) {
    double W[NEQ_MAX], U[NEQ_MAX];
    for (int v = 0; v < neq; ++v) U[v] = q[v * nc + c];
    cell_cons_to_prim(P, U, W);
    for (int v = 0; v < neq; ++v) w[v * nc + c] = W[v];
  }
  return ORC_OK;
}

/* Mixture sound speed squared at every cell (diagnostic). */
int orc_sound_speed_sq(const orc_problem* P, const double* q, double* c2) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P), nf = P->num_fluids;
  int64_t nc = ncell(P);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c) {
    double U[NEQ_MAX], W[NEQ_MAX];
    for (int v = 0; v < neq; ++v) U[v] = q[v * nc + c];
    cell_cons_to_prim(P, U, W);
    double rho = 0.0;
    for (int i = 0; i < nf; ++i) rho = rho + U[i];
    double Gam, Pi;
    mixture(P, nf == 2 ? &U[row_alpha(P, 0)] : NULL, &Gam, &Pi);
    c2[c] = sound_speed_sq(rho, W[row_E(P)], Gam, Pi);
  }
  return ORC_OK;
}

/* Conservation sums: sum over cells of each row, times the cell volume.
 * Accumulated in long double for accuracy (diagnostic only). */
int orc_conserved_sums(const orc_problem* P, const double* q, double* sums) {
  if (orc_validate(P)) return ORC_ERR_ARG;
  int neq = orc_num_eqs(P);
  int64_t nc = ncell(P);
  int uniform = !P->faces[0] && !P->faces[1] && !P->faces[2];
  double vol = 1.0;
  for (int d = 0; d < P->ndim; ++d) vol = vol * P->dx[d];
  for (int v = 0; v < neq; ++v) {
    long double acc = 0.0L;
    if (uniform) {
      for (int64_t c = 0; c < nc; ++c) acc += (long double)q[v * nc + c];
      sums[v] = (double)acc * vol;
    } else {
      /* non-uniform grid: each cell's own volume */
      for (int64_t c = 0; c < nc; ++c) {
        int idx[3] = {(int)(c % P->n[0]), (int)((c / P->n[0]) % P->n[1]),
                      (int)(c / ((int64_t)P->n[0] * P->n[1]))};
        long double cv = 1.0L;
        for (int d = 0; d < P->ndim; ++d) cv *= (long double)cell_width(P, d, idx[d]);
        acc += (long double)q[v * nc + c] * cv;
      }
      sums[v] = (double)acc;
    }
  }
  return ORC_OK;
}

int orc_abi_version(void) { return 1; }

/* Set the OpenMP thread count of the parallel loops (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* OpenMP threads the parallel loops use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
