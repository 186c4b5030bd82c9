// Grouped specialised FFT passes of length 100 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_GROUP_INSTANTIATE(100)
}  // namespace vg
