// Specialised row passes of length 2048 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(2048, true)
}  // namespace vg
