// sweep_wv3.hip -- axis passes with WENO5-M reconstruction.
#include "sweep_impl.h"

namespace mfc {
MFC_INSTANTIATE_SWEEP(3)
}  // namespace mfc
