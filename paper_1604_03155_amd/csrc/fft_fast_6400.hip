// Specialised row passes of length 6400 (see fft_fast_impl.h): the rows of the
// 2D grids N = 3200 used in the paper's 2D scattering runs (Tables 4-6).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(6400, true)
}  // namespace vg
