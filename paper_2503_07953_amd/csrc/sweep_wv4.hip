// sweep_wv4.hip -- axis passes with WENO5-JS on a non-uniform grid
// (tabulated candidates, indicators and ideal weights; Sec. 4.2.2).
#include "sweep_impl.h"

namespace mfc {
MFC_INSTANTIATE_SWEEP(4)
}  // namespace mfc
