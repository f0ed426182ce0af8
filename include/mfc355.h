/*
 * mfc355.h -- C ABI of the MI355X (gfx950) five-equation right-hand side.
 *
 * The library evaluates the semi-discrete right-hand side of the
 * five-equation diffuse-interface model (arXiv 2503.07953, Sec. 2.1.1, eq.
 * five_eqn_transport; Allaire form with K = 0 by default, Kapila's K as an
 * option) closed by the stiffened-gas equation of state (Sec. 2.2, eq. eos),
 * on a structured grid (uniform, or non-uniform per axis, Sec. 4.2.2), and
 * advances it with the three-stage SSP Runge-Kutta scheme (Sec. 3.4):
 *
 *   dq_{ijk}/dt = sum_d (F_{-1/2} - F_{+1/2})/dx_d + alpha (div u)_{ijk}
 *
 * (eq. eqn:rhs with s = 0 and h = -alpha), with face fluxes from WENO5-JS
 * reconstruction of primitive variables (Sec. 3.2.1) and the HLLC solver
 * (Sec. 3.2.2), which also returns the face velocity used for div u; other
 * reconstruction weights, face solvers and low-Mach treatments are options.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Arrays: caller-owned DEVICE memory, structure-of-arrays, C order
 *   q[v][k][j][i] (x fastest), interior cells only, element type given by
 *   mfc_problem.precision (double for MFC_FP64, float for MFC_FP32_MIXED),
 *   aligned to the element size.  Rows for nf fluids in D dimensions:
 *     alpha_i rho_i (nf rows), rho u_d (D rows), rho E,
 *     alpha_i (nf rows, only for nf == 2).
 *   mfc_num_eqs() gives the row count.  Primitive arrays use the rows
 *   alpha_i rho_i, u_d, p, alpha_i.  Scalars returned on the device
 *   (dt, signal speed, sums) are always double.
 * Ownership: the library never frees or keeps user pointers after a call
 *   returns; the context owns only its own scratch.
 * Streams: every call is asynchronous on `hip_stream` (a hipStream_t; NULL
 *   is the default stream).  A context serves one stream at a time.
 * Devices: a context belongs to the HIP device that was current at
 *   mfc_create; every later call must be made with that device current
 *   (MFC_ERR_ARG otherwise), and every array must live on it.
 * Errors: negative return codes.  Argument, shape and alignment checks run on
 *   the host before any HIP call.  Launch failures return MFC_ERR_HIP.  A
 *   face state with non-positive squared sound speed or a non-finite flux
 *   sets a device flag that mfc_check() reports as MFC_ERR_NONFINITE.
 *   mfc_last_error() describes the last failure of a context.
 */
#ifndef MFC355_H
#define MFC355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFC_ABI_VERSION 5

enum {
  MFC_OK = 0,
  MFC_ERR_ARG = -1,         /* null pointer, bad value, misaligned pointer */
  MFC_ERR_SHAPE = -2,       /* grid sizes inconsistent with ndim or too large */
  MFC_ERR_UNSUPPORTED = -3, /* ndim, fluid count or precision not provided */
  MFC_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed */
  MFC_ERR_NONFINITE = -5,   /* c^2 <= 0 or a non-finite flux was met */
  MFC_ERR_ALLOC = -6        /* device scratch allocation failed */
};

/* Boundary conditions through three ghost layers per side (Sec. 3.3):
 * PERIODIC wraps (both sides of an axis must be periodic); EXTRAP copies the
 * nearest interior cell; SLIPWALL mirrors the interior with the wall-normal
 * momentum negated. */
enum { MFC_BC_PERIODIC = 0, MFC_BC_EXTRAP = 1, MFC_BC_SLIPWALL = 2 };

/* MFC_FP64: double storage and arithmetic.
 * MFC_FP32_MIXED: float storage, float WENO/HLLC arithmetic; double for the
 * pressure inversion from total energy, sound and wave speeds, the stage
 * combination, the CFL reduction and the conservation sums. */
enum { MFC_FP64 = 0, MFC_FP32_MIXED = 1 };

/* Reconstruction weights, all on the same three candidates, smoothness
 * indicators, linear weights d_k and eps:
 *   MFC_WENO_JS  Jiang-Shu, d_k/(eps + beta_k)^2 (Sec. 3.2.1);
 *   MFC_WENO_M   the Jiang-Shu weights w_k mapped by Henrick, Aslam and
 *                Powers' g_k(w) = w (d_k + d_k^2 - 3 d_k w + w^2) /
 *                (d_k^2 + w (1 - 2 d_k)) and normalized again (Sec. 3.2.1,
 *                which names the mapping without printing it);
 *   MFC_WENO_Z   d_k (1 + tau/(beta_k + eps)), tau = |beta_0 - beta_2|, q = 1
 *                (Sec. 4.2.2);
 *   MFC_TENO     stencil k kept when its share of gamma_k =
 *                d_k (1 + tau/(beta_k + eps))^6 reaches C_T = 1e-5, kept
 *                stencils weighted d_k (Sec. 4.2.2; the cut-off is not printed
 *                there: the published fifth-order value). */
enum { MFC_WENO_JS = 0, MFC_WENO_Z = 1, MFC_TENO = 2, MFC_WENO_M = 3 };

/* Face solver (Sec. 3.2.2; Toro's book):
 *   MFC_HLLC  three waves, star states from continuity of normal velocity and
 *             pressure; the volume fractions ride the contact;
 *   MFC_HLL   two waves and one averaged state, F = (S_R F_L - S_L F_R +
 *             S_L S_R (U_R - U_L))/(S_R - S_L) between them; the volume
 *             fractions take the same formula on alpha u_n and the face
 *             velocity of the alpha source is (S_R u_L - S_L u_R)/(S_R - S_L)
 *             (the paper prints no HLL formula: these are the readings). */
enum { MFC_HLLC = 0, MFC_HLL = 1 };

/* Low-Mach treatment (the paper's low-Mach section, Sec. 4.2.4), with
 * z = min(max(|u_L|/c_L, |u_R|/c_R), 1) from the face states as reconstructed:
 *   MFC_LOW_MACH_NONE      the face states as reconstructed;
 *   MFC_LOW_MACH_THORNBER  Thornber et al.: the face-normal velocities become
 *                          (u_L + u_R)/2 +- z (u_L - u_R)/2 before the face
 *                          solver (either one);
 *   MFC_LOW_MACH_CHEN_APC  Chen et al.: the anti-dissipation pressure
 *                          correction (z - 1) p_d on the normal-momentum flux
 *                          and (z - 1) p_d S* on the energy flux of both HLLC
 *                          star regions, p_d = rho_L rho_R (S_L - u_L)
 *                          (S_R - u_R)(u_R - u_L) / (rho_R (S_R - u_R) -
 *                          rho_L (S_L - u_L)); HLLC only. */
enum { MFC_LOW_MACH_NONE = 0, MFC_LOW_MACH_THORNBER = 1, MFC_LOW_MACH_CHEN_APC = 2 };

/* Five-equation model (Sec. 2.1.1):
 *   MFC_MODEL_ALLAIRE  K = 0: the alpha_i rows carry alpha_i div u;
 *   MFC_MODEL_KAPILA   the alpha_1 row carries (alpha_1 + K) div u and the
 *                      alpha_2 row (alpha_2 - K) div u, K = (rho_2 c_2^2 -
 *                      rho_1 c_1^2) / (rho_1 c_1^2/alpha_1 + rho_2 c_2^2/alpha_2),
 *                      phasic c_i^2 = gamma_i (p + pi_inf,i)/rho_i, from each
 *                      cell's average state.  The paper prints a plus sign in
 *                      the numerator; the difference is read, since only it
 *                      vanishes for two identical fluids.  Two fluids only. */
enum { MFC_MODEL_ALLAIRE = 0, MFC_MODEL_KAPILA = 1 };

typedef struct {
  int32_t abi_version; /* must equal MFC_ABI_VERSION */
  int32_t ndim;        /* 1, 2 or 3 */
  int32_t n[3];        /* interior cells per axis; >= 3 on active axes, 1 on unused;
                          n[1], n[2] <= 65535, n[0]*n[1]*n[2] <= 2^34 */
  int32_t num_fluids;  /* 1 (Euler) or 2 (five-equation model) */
  int32_t precision;   /* MFC_FP64 or MFC_FP32_MIXED */
  int32_t bc_lo[3];    /* MFC_BC_* per axis, low side */
  int32_t bc_hi[3];    /* MFC_BC_* per axis, high side */
  double dx[3];        /* uniform spacing per axis (> 0 on active axes) */
  double gamma[2];     /* stiffened-gas gamma_i > 1 per fluid (Sec. 2.2) */
  double pi_inf[2];    /* stiffened-gas pi_inf,i >= 0 per fluid */
  double weno_eps;     /* WENO smoothness regularization, 1e-30 <= eps < 1e300
                          (1e-6); smaller values are rejected with MFC_ERR_ARG
                          because the double reconstruction normalizes through
                          a product of eight terms of size >= 4 eps */
  int32_t weno_variant; /* MFC_WENO_JS, MFC_WENO_Z, MFC_TENO or MFC_WENO_M */
  int32_t riemann_solver; /* MFC_HLLC (0) or MFC_HLL */
  int32_t low_mach;       /* MFC_LOW_MACH_NONE (0), _THORNBER or _CHEN_APC (HLLC only) */
  int32_t model;          /* MFC_MODEL_ALLAIRE (0) or MFC_MODEL_KAPILA (two fluids) */
} mfc_problem;

typedef struct mfc_ctx mfc_ctx;

/* Library and problem queries (host only, no HIP calls). */
int mfc_abi_version(void);
const char* mfc_status_string(int status);
/* Row count: 2N + D + 1 for two fluids, D + 2 for one; negative on error. */
int mfc_num_eqs(const mfc_problem* prob);
/* Full host-side validation of a problem description; MFC_OK or an error. */
int mfc_validate(const mfc_problem* prob);

/* Create a context for `prob` on the current HIP device: validates, copies the
 * description and allocates device scratch (two stage states, one RHS
 * accumulator, reduction partials and flags).  *out is NULL on failure. */
int mfc_create(const mfc_problem* prob, mfc_ctx** out);
/* Release a context and its scratch (synchronizes the device).  NULL is a no-op. */
int mfc_destroy(mfc_ctx* ctx);
/* Description of the last error met by `ctx` (never NULL). */
const char* mfc_last_error(const mfc_ctx* ctx);

/* Primitive (alpha_i rho_i, u_d, p, alpha_i) -> conservative rows with the
 * mixture rule rho E = Gamma p + Pi + rho |u|^2 / 2 (Sec. 2.1.1, 2.2).
 * w and q may not alias. */
int mfc_prim_to_cons(mfc_ctx* ctx, const void* w, void* q, void* hip_stream);
/* Conservative -> primitive: u_d = (rho u_d)/rho, p = (rho E - rho|u|^2/2 - Pi)/Gamma. */
int mfc_cons_to_prim(mfc_ctx* ctx, const void* q, void* w, void* hip_stream);

/* Right-hand side L(q) of eq. eqn:rhs: rhs = sum over axes of the flux
 * difference plus alpha (u_{+1/2} - u_{-1/2})/dx on the alpha rows.
 * q and rhs: neq*ncell elements; they may not alias. */
int mfc_rhs(mfc_ctx* ctx, const void* q, void* rhs, void* hip_stream);

/* Largest signal speed s = max_cells sum_d (|u_d| + c)/dx_d (the time-step
 * rule; the paper states none) written to smax_dev (device double). */
int mfc_max_signal(mfc_ctx* ctx, const void* q, double* smax_dev, void* hip_stream);

/* One SSP-RK3 step (Shu-Osher form, Sec. 3.4), in place: q holds q^n on entry
 * and q^{n+1} on return.  Exactly one of `cfl` (> 0: dt = cfl/s computed on
 * the device from q^n, clipped to t_remaining when t_remaining > 0) and
 * `dt_fixed` (> 0) must be positive, else MFC_ERR_ARG.  dt_dev (device
 * double, may be NULL) receives the dt used.  No host synchronization. */
int mfc_step(mfc_ctx* ctx, void* q, double cfl, double dt_fixed, double t_remaining,
             double* dt_dev, void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The step of
 * mfc_step (same kernels, same results bit for bit) without a context: the
 * RHS accumulator, both stage states, the reduction partials and [smax, dt]
 * live in one static device array of MFC_STATIC_SCRATCH_BYTES per GPU, held
 * from the first call on a device until the process ends.  Nothing is
 * allocated and no memset is issued.
 *   prob      validated as by mfc_validate (its code is returned on failure);
 *   q         caller's device state (layout as mfc_step), advanced in place;
 *   cfl, dt_fixed, t_remaining, dt_dev: as mfc_step;
 *   flag_dev  caller's device int (required): set to nonzero when c^2 <= 0 or
 *             a non-finite flux is met, never cleared by the library.
 * Size limit: 3 * round256(neq * ncell * sizeof(element)) + round256(8 *
 * max(8192, blocks of the first axis pass)) + 256 bytes must fit
 * MFC_STATIC_SCRATCH_BYTES (about 1.3M cells for 3D two-fluid FP64, 2.7M in
 * FP32), else MFC_ERR_SHAPE before any HIP call.  MFC_ERR_HIP if a launch
 * fails or the array's address cannot be resolved.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (other streams, other threads) race.
 * The call keeps nothing from an earlier call. */
#define MFC_STATIC_SCRATCH_BYTES (256u << 20)
int mfc_step_static(const mfc_problem* prob, void* q, double cfl, double dt_fixed, double t_remaining,
                    double* dt_dev, int* flag_dev, void* hip_stream);

/* Non-uniform grid along `axis` (Sec. 4.2.2): faces is a HOST array of the
 * n[axis] + 1 cell-face coordinates x_{-1/2} .. x_{n-1/2}, strictly
 * increasing and finite (read during the call, not kept); NULL restores the
 * uniform spacing dx[axis].  Cell i then has width h_i = x_{i+1/2} -
 * x_{i-1/2}, which replaces dx in the flux difference, the alpha source, the
 * signal speed and the conservation sums (cell volume h_x h_y h_z).  The
 * fifth-order reconstruction on the grid: in the unit coordinate of each
 * centre cell, candidate r is the quadratic with the stencil's data as its
 * cell averages, its smoothness indicator is sum_{l=1,2} h^(2l-1)
 * int_cell (d^l p/dx^l)^2 dx, and the ideal weights at each face are those
 * that combine the candidates into the quartic with the five cells' averages
 * (the paper states the candidates and indicators; these weights are the
 * reading).  Ghost cells take the width of the cell whose state they hold
 * (wrap, nearest cell or mirror image).  The coefficients are formed on the
 * host in double and kept on the device in the context (allocated at the
 * first call, synchronous copy).
 * WENO5-JS problems only (MFC_ERR_UNSUPPORTED otherwise); the adjoint entry
 * points follow the grid (their hand-written VJP of the tabulated
 * reconstruction and per-cell widths); mfc_step_static (no context) always
 * uses the uniform spacing.
 * MFC_ERR_ARG for a bad axis or face array. */
int mfc_set_grid(mfc_ctx* ctx, int axis, const double* faces);

/* Conservation diagnostics: sums_dev[v] =(sum over cells of q[v]) * cell volume,
 * neq device doubles, accumulated in double with a fixed reduction order. */
int mfc_conserved_sums(mfc_ctx* ctx, const void* q, double* sums_dev, void* hip_stream);

/* ---- Discrete adjoint (FP64 contexts only; MFC_ERR_UNSUPPORTED otherwise) ----
 * Hand-written reverse mode of the discrete operators above (not in the paper,
 * which has no adjoint): derivatives follow the branch the forward pass takes
 * (wave-speed min/max ties to the first argument, HLLC region order as in the
 * forward solver).  The first call allocates adjoint scratch in the context:
 * 6*neq+1 doubles per face of every axis when that sum is at most 8 GiB (all
 * axes' face passes then run as one launch), else per face of the largest
 * axis only, plus three states.  The environment variable
 * MFC355_ADJOINT_FACE_BUDGET (bytes, read at that first call) overrides the
 * 8 GiB threshold.
 * Outputs may not alias inputs.  accumulate != 0 adds to the output instead of
 * overwriting it.  Both face solvers (HLLC, HLL) and the low-Mach correction
 * have their hand-written adjoint. */

/* q_bar (+)= (dL/dq)^T rhs_bar, L the right-hand side of mfc_rhs at q. */
int mfc_rhs_vjp(mfc_ctx* ctx, const void* q, const void* rhs_bar, void* q_bar, int accumulate,
                void* hip_stream);

/* Adjoint of one SSP-RK3 step with the fixed time step dt (a frozen-dt step,
 * as mfc_step with dt_fixed = dt): qn_bar = (dq^{n+1}/dq^n)^T qnp1_bar.  The
 * stage states are recomputed from q_n inside the call. */
int mfc_step_vjp(mfc_ctx* ctx, const void* q_n, double dt, const void* qnp1_bar, void* qn_bar,
                 void* hip_stream);

/* The fixed-dt SSP-RK3 step of mfc_step (q advanced in place) that also writes
 * its two stage states, q1 = q + dt L(q) and q2 = 3/4 q + 1/4 (q1 + dt L(q1))
 * (Sec. 3.4), to the caller's arrays q1 and q2 (same layout as q, distinct from
 * q and from each other).  Used to replay a checkpointed segment once and hand
 * its stages to mfc_step_vjp_stages.  FP64 contexts. */
int mfc_step_save_stages(mfc_ctx* ctx, void* q, double dt, void* q1, void* q2, void* hip_stream);

/* mfc_step_vjp with the stage states of the step from q_n supplied (as written
 * by mfc_step_save_stages for the same q_n and dt), so that they are not
 * recomputed.  qn_bar must alias none of the inputs. */
int mfc_step_vjp_stages(mfc_ctx* ctx, const void* q_n, const void* q1, const void* q2, double dt,
                        const void* qnp1_bar, void* qn_bar, void* hip_stream);

/* q_bar (+)= (dw/dq)^T w_bar for the conversion of mfc_cons_to_prim at q. */
int mfc_cons_to_prim_vjp(mfc_ctx* ctx, const void* q, const void* w_bar, void* q_bar, int accumulate,
                         void* hip_stream);

/* w_bar (+)= (dq/dw)^T q_bar for the conversion of mfc_prim_to_cons at w. */
int mfc_prim_to_cons_vjp(mfc_ctx* ctx, const void* w, const void* q_bar, void* w_bar, int accumulate,
                         void* hip_stream);

/* Synchronize `hip_stream`, then report and clear the non-finite flag:
 * MFC_OK or MFC_ERR_NONFINITE (or MFC_ERR_HIP if the stream failed). */
int mfc_check(mfc_ctx* ctx, void* hip_stream);

/* Diagnostics: launch timing.  While enabled, every kernel launch of
 * mfc_step, mfc_rhs and the VJP entry points is bracketed by a pair of HIP
 * events recorded on its own launch stream.  mfc_get_timing waits for the
 * recorded events and returns, per launch kind
 *   0 signal-speed reduction, 1 x pass, 2 y pass, 3 z pass, 4 adjoint passes,
 * the summed milliseconds (ms_sum[5]) and launch counts (counts[5]) since the
 * previous call, then starts a new interval.  Timing adds two event records
 * per launch; it is off after mfc_create. */
#define MFC_TIMING_KINDS 5
int mfc_set_timing(mfc_ctx* ctx, int enable);
int mfc_get_timing(mfc_ctx* ctx, double* ms_sum, int64_t* counts);

#ifdef __cplusplus
}
#endif
#endif /* MFC355_H */
