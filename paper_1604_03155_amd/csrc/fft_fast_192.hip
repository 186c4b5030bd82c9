// Specialised FFT passes of length 192 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(192, false)
}  // namespace vg
