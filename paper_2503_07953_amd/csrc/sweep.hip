// sweep.hip -- dispatch of the fused axis passes over the reconstruction
// variants (each instantiated in its own sweep_wv*.hip), and the signal
// partials length of the first pass.
#include "sweep_impl.h"

namespace mfc {

MFC_EXTERN_SWEEP(0)
MFC_EXTERN_SWEEP(1)
MFC_EXTERN_SWEEP(2)
MFC_EXTERN_SWEEP(3)
MFC_EXTERN_SWEEP(4)

long long signal_partials(int ndim, const int* n) {
  if (ndim == 2) {
    const long long a = first_pass_blocks<2, double>(n), b = first_pass_blocks<2, float>(n);
    return a > b ? a : b;
  }
  if (ndim == 3) {
    const long long a = first_pass_blocks<3, double>(n), b = first_pass_blocks<3, float>(n);
    return a > b ? a : b;
  }
  return 0;
}

template <typename Real>
hipError_t launch_rhs(int nf, int ndim, const Params& pm, const Real* qk, Real* acc, const Real* qn,
                      Real* qout, StageArgs st, bool final_step, int* flag, hipStream_t s, PassTimer* tm,
                      const SignalFuse* sig) {
  if (pm.nu[0] || pm.nu[1] || pm.nu[2])
    return launch_rhs_wv<kWvNonUniform, Real>(nf, ndim, pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
  switch (pm.weno_variant) {
    case 1: return launch_rhs_wv<1, Real>(nf, ndim, pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
    case 2: return launch_rhs_wv<2, Real>(nf, ndim, pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
    case 3: return launch_rhs_wv<3, Real>(nf, ndim, pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
    default: return launch_rhs_wv<0, Real>(nf, ndim, pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
  }
}

template hipError_t launch_rhs<double>(int, int, const Params&, const double*, double*, const double*,
                                       double*, StageArgs, bool, int*, hipStream_t, PassTimer*,
                                       const SignalFuse*);
template hipError_t launch_rhs<float>(int, int, const Params&, const float*, float*, const float*, float*,
                                      StageArgs, bool, int*, hipStream_t, PassTimer*, const SignalFuse*);

}  // namespace mfc
