// vjp_wv4.hip -- RHS adjoint passes with WENO5-JS on a non-uniform grid.
#include "vjp_impl.h"

namespace mfc {
MFC_INSTANTIATE_VJP(4)
}  // namespace mfc
