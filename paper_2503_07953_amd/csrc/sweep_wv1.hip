// sweep_wv1.hip -- axis passes with WENO5-Z reconstruction.
#include "sweep_impl.h"

namespace mfc {
MFC_INSTANTIATE_SWEEP(1)
}  // namespace mfc
