// sweep_wv0.hip -- axis passes with WENO5-JS reconstruction.
#include "sweep_impl.h"

namespace mfc {
MFC_INSTANTIATE_SWEEP(0)
}  // namespace mfc
