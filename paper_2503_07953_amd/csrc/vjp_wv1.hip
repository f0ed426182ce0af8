// vjp_wv1.hip -- RHS adjoint passes with WENO5-Z reconstruction.
#include "vjp_impl.h"

namespace mfc {
MFC_INSTANTIATE_VJP(1)
}  // namespace mfc
