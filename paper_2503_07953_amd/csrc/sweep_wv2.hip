// sweep_wv2.hip -- axis passes with TENO5 reconstruction.
#include "sweep_impl.h"

namespace mfc {
MFC_INSTANTIATE_SWEEP(2)
}  // namespace mfc
