// Specialised row passes of length 3200 (see fft_fast_impl.h): the rows of the
// 2D grids N = 1600 used in the paper's 2D scattering runs (Tables 4-6).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(3200, true)
}  // namespace vg
