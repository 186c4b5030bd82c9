// Specialised FFT passes of length 128 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(128, false)
}  // namespace vg
