// vjp_wv0.hip -- RHS adjoint passes with WENO5-JS reconstruction.
#include "vjp_impl.h"

namespace mfc {
MFC_INSTANTIATE_VJP(0)
}  // namespace mfc
