// internal.h -- host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mfc {

// Output mode of an axis pass.  MODE_SIGNAL (with MODE_WRITE, on the first
// pass of a CFL step's first stage) also forms the block maxima of the signal
// speed of every loaded cell.
enum { MODE_WRITE = 0, MODE_ACC = 1, MODE_STEP = 2, MODE_SIGNAL = 4 };

// Stage description for the fused SSP-RK3 combination.
struct StageArgs {
  int stage;              // 1, 2 or 3
  double dt;              // used when dt_ptr is null
  const double* dt_ptr;   // device dt (CFL steps)
  double* sig_partial;    // MODE_SIGNAL: one maximum per block of the pass
};

// CFL time step formed inside the first RHS evaluation of a step (2D and 3D):
// the first axis pass writes per-block signal maxima to `partial`, then one
// block forms smax, dt = cfl/smax (clipped to t_remaining when > 0) and
// writes them to smax_out, dt_out and (if not null) dt_user.
struct SignalFuse {
  double* partial;
  double cfl;
  double t_remaining;
  double* smax_out;
  double* dt_out;
  double* dt_user;
};

// Internal reconstruction variant of the axis passes on a non-uniform grid
// (WENO5-JS with tabulated coefficients); 0..3 are the uniform variants.
constexpr int kWvNonUniform = 4;

// Compile-time option bits of a problem (RS_HLL, RS_THORNBER, RS_APC, RS_KAPILA).
inline int option_bits(const Params& pm) {
  return (pm.riemann == 1 ? RS_HLL : 0) | (pm.low_mach == 1 ? RS_THORNBER : 0) | (pm.low_mach == 2 ? RS_APC : 0) |
         (pm.model == 1 ? RS_KAPILA : 0);
}

// Kinds of timed launches (see mfc_set_timing).
enum { KIND_SIGNAL = 0, KIND_PASS_X = 1, KIND_PASS_Y = 2, KIND_PASS_Z = 3, KIND_VJP = 4, KIND_COUNT = 5 };

// Optional hook that brackets every launch of an entry point with events on
// the launch stream.
struct PassTimer {
  virtual void begin(int kind, hipStream_t s) = 0;
  virtual void end(int kind, hipStream_t s) = 0;
  virtual ~PassTimer() {}
};

// Number of blocks of the fixed-shape reductions (partials buffer length).
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

template <typename Real>
hipError_t launch_rhs(int nf, int ndim, const Params& pm, const Real* qk, Real* acc, const Real* qn,
                      Real* qout, StageArgs st, bool final_step, int* flag, hipStream_t s,
                      PassTimer* tm = nullptr, const SignalFuse* sig = nullptr);

// Length of the partials buffer that SignalFuse needs for a grid (the block
// count of the first axis pass; 0 in 1D, where the signal is a kernel of its own).
long long signal_partials(int ndim, const int* n);

hipError_t launch_finalize_dt(const double* partial, int nparts, double cfl, double t_remaining, double* smax_out,
                              double* dt_out, double* dt_user, hipStream_t s);

template <typename Real>
hipError_t launch_max_signal(int nf, int ndim, const Params& pm, const Real* q, double* partial,
                             double* smax_out, double cfl, double t_remaining, double* dt_out,
                             double* dt_user, int* flag, hipStream_t s);

template <typename Real>
hipError_t launch_sums(int neq, const Params& pm, const Real* q, double vol, double* partial,
                       double* sums_out, hipStream_t s);

template <typename Real>
hipError_t launch_convert(int nf, int ndim, bool to_cons, const Params& pm, const Real* in, Real* out,
                          hipStream_t s);

hipError_t launch_set_scalar(double* dst, double value, hipStream_t s);

// Scratch of the adjoint passes (owned by the context, allocated on first use).
// all_axes: one face buffer per axis (Gd[d], UFd[d]) so that the face passes of
// every axis run in one launch; otherwise only Gd[0] / UFd[0] exist and the
// axes are processed one after the other.
struct VjpScratch {
  double* Gd[3];    // per-face primitive cotangents of the 6 stencil positions
  double* UFd[3];   // per-face forward face velocity
  bool all_axes;
};

// Reverse SSP-RK3 stage combination applied to v = L^T rbar as the cell pass
// writes it (stage 0: none, qbar = v or qbar += v):
//   stage 3: out = 2/3 (x + dt v), qnb = x / 3
//   stage 2: out = 1/4 (x + dt v), qnb += 3/4 x
//   stage 1: qnb += x + dt v
struct StageEpi {
  int stage;
  double dt;
  const double* x;
  double* out;
  double* qnb;
};
// epi (stage > 0, accumulate false) is applied in the cell pass when every
// axis is gathered in one pass (sc.all_axes), in place of writing qbar; with
// the axes one after the other (!sc.all_axes) it is ignored, qbar is written,
// and the caller applies the combination (launch_adj_stage).
hipError_t launch_rhs_vjp(int nf, int ndim, const Params& pm, const double* q, const double* rbar, double* qbar,
                          const VjpScratch& sc, bool accumulate, hipStream_t s, PassTimer* tm,
                          const StageEpi* epi = nullptr);
hipError_t launch_convert_vjp(int nf, int ndim, bool to_cons, const Params& pm, const double* x, const double* ybar,
                              double* xbar, bool accumulate, hipStream_t s);
hipError_t launch_adj_stage(int which, long long n, double dt, const double* x, const double* v, double* out,
                            double* qnb, hipStream_t s);

}  // namespace mfc
