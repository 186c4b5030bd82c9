// Specialised row passes of length 12800 (see fft_fast_impl.h): the rows of the
// 2D grid N = 6400 of the paper's largest 2D scattering runs (Table 4); a
// complex64 row (100 KiB) is exchanged as real and imaginary parts in turn.
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(12800, true)
}  // namespace vg
