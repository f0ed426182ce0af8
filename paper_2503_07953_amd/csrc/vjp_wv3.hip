// vjp_wv3.hip -- RHS adjoint passes with WENO5-M reconstruction.
#include "vjp_impl.h"

namespace mfc {
MFC_INSTANTIATE_VJP(3)
}  // namespace mfc
