// Specialised FFT passes of length 96 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(96, false)
}  // namespace vg
