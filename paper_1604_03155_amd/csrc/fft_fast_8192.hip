// Specialised row passes of length 8192 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(8192, true)
}  // namespace vg
