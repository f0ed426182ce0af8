// vjp_wv2.hip -- RHS adjoint passes with TENO5 reconstruction.
#include "vjp_impl.h"

namespace mfc {
MFC_INSTANTIATE_VJP(2)
}  // namespace mfc
