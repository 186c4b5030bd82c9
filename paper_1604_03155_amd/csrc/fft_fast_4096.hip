// Specialised row passes of length 4096 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(4096, true)
}  // namespace vg
